// Many small partial SVDs at once: locally low-rank models (Sec. I and
// Sec. V point out that the batched small eigen-problems at the heart of the
// method serve these as well).
//
// For B Casorati matrices X_b (m rows, e.g. the pixels of a patch; Q columns,
// e.g. channels or frames), the r largest singular values and right
// singular vectors come from the Gram A_b = X_b^H X_b (Q x Q, Hermitian,
// formed in FP32): its r largest eigenpairs are the r smallest of -A_b,
// found by the per-voxel Lanczos solver with a full Krylov basis; sigma_k =
// sqrt(lambda_k).  The rank-r part X_b V V^H (the truncated SVD, Eckart-Young)
// is formed last.  The Gram route resolves sigma_k to about
// eps sigma_1^2 / sigma_k.
//
// The Grams are dense contractions (8 m Q(Q+1)/2 flops per patch) and run on
// the FP32 matrix cores, one wave per patch; the projection is bound by its
// read of X and write of the result.
#include "common.hpp"

namespace pisco {

typedef float f32x4 __attribute__((ext_vector_type(4)));

// -A_b packed upper, voxel-major [B][Q(Q+1)/2] (each patch's entries
// contiguous, as the Lanczos kernel reads them); X is [B][Q][m].
// One wave per patch on FP32 matrix cores (v_mfma_f32_16x16x4f32): the
// Hermitian Gram as 16 x 16 channel blocks (0,0), (0,1), (1,1) (one block
// for Q <= 16), Re = Xr^T Xr + Xi^T Xi and Im = Xr^T Xi - Xi^T Xr.  The patch
// goes through LDS in chunks of 32 pixels, loaded one coalesced row segment
// per instruction; lane (li, kg) = (l % 16, l / 16) then supplies channels li
// and 16 + li at pixel 8 kg + s of step s.  A and B of a product are the same
// lane values, since both sides of the Gram are columns of X at one pixel.
template <int NQB>
__global__ void __launch_bounds__(64) k_llr_gram(const float2* __restrict__ X,
                                                 float2* __restrict__ A, long long B, int Q,
                                                 int m, unsigned* status) {
  constexpr int kC = 32;  // pixels per chunk
  __shared__ float2 tile[16 * NQB][kC + 1];
  const long long b = xcd_block(blockIdx.x, gridDim.x);
  if (b >= B) return;
  const int l = threadIdx.x, li = l & 15, kg = l >> 4;
  const float2* xb = X + size_t(b) * Q * m;
  f32x4 cr[3], ci[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    cr[k] = f32x4{0.f, 0.f, 0.f, 0.f};
    ci[k] = f32x4{0.f, 0.f, 0.f, 0.f};
  }
  bool bad = false;
  for (int i0 = 0; i0 < m; i0 += kC) {
    // rows 2t and 2t + 1 of the chunk per instruction (zeros past Q and m)
#pragma unroll
    for (int t = 0; t < 8 * NQB; ++t) {
      const int q = 2 * t + (l >> 5), i = i0 + (l & 31);
      float2 xv = make_float2(0.f, 0.f);
      if (q < Q && i < m) xv = xb[size_t(q) * m + i];
      bad |= !isfinite(xv.x) || !isfinite(xv.y);
      tile[q][l & 31] = xv;
    }
    wave_sync();
#pragma unroll
    for (int s = 0; s < kC / 4; ++s) {
      const float2 x0 = tile[li][8 * kg + s];
      // block (0,0)
      cr[0] = __builtin_amdgcn_mfma_f32_16x16x4f32(x0.x, x0.x, cr[0], 0, 0, 0);
      ci[0] = __builtin_amdgcn_mfma_f32_16x16x4f32(x0.x, x0.y, ci[0], 0, 0, 0);
      cr[0] = __builtin_amdgcn_mfma_f32_16x16x4f32(x0.y, x0.y, cr[0], 0, 0, 0);
      ci[0] = __builtin_amdgcn_mfma_f32_16x16x4f32(-x0.y, x0.x, ci[0], 0, 0, 0);
      if (NQB == 2) {
        // blocks (0,1) and (1,1)
        const float2 x1 = tile[16 + li][8 * kg + s];
        cr[1] = __builtin_amdgcn_mfma_f32_16x16x4f32(x0.x, x1.x, cr[1], 0, 0, 0);
        ci[1] = __builtin_amdgcn_mfma_f32_16x16x4f32(x0.x, x1.y, ci[1], 0, 0, 0);
        cr[2] = __builtin_amdgcn_mfma_f32_16x16x4f32(x1.x, x1.x, cr[2], 0, 0, 0);
        ci[2] = __builtin_amdgcn_mfma_f32_16x16x4f32(x1.x, x1.y, ci[2], 0, 0, 0);
        cr[1] = __builtin_amdgcn_mfma_f32_16x16x4f32(x0.y, x1.y, cr[1], 0, 0, 0);
        ci[1] = __builtin_amdgcn_mfma_f32_16x16x4f32(-x0.y, x1.x, ci[1], 0, 0, 0);
        cr[2] = __builtin_amdgcn_mfma_f32_16x16x4f32(x1.y, x1.y, cr[2], 0, 0, 0);
        ci[2] = __builtin_amdgcn_mfma_f32_16x16x4f32(-x1.y, x1.x, ci[2], 0, 0, 0);
      }
    }
    wave_sync();  // the next chunk overwrites the tile
  }
  if (bad) atomicOr(status, PISCO_FLAG_NONFINITE);
  // lane (li, kg) holds D[4 kg + r][li] of each block
#pragma unroll
  for (int bk = 0; bk < (NQB == 2 ? 3 : 1); ++bk) {
    const int pb = bk == 2 ? 1 : 0, qb = bk == 0 ? 0 : 1;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int p = 16 * pb + 4 * kg + r, q = 16 * qb + li;
      if (p <= q && q < Q) {
        const int pair = p * Q - p * (p - 1) / 2 + (q - p);
        A[size_t(b) * (Q * (Q + 1) / 2) + pair] =
            p == q ? make_float2(-cr[bk][r], 0.f) : make_float2(-cr[bk][r], -ci[bk][r]);
      }
    }
  }
}

// sigma = sqrt(max(lambda(A), 0)) from the eigenvalues of -A
__global__ void k_llr_sigma(const float* __restrict__ lamneg, float* __restrict__ sigma,
                            long long n) {
  const long long i = blockIdx.x * 256LL + threadIdx.x;
  if (i < n) sigma[i] = sqrtf(fmaxf(-lamneg[i], 0.f));
}

// Xr_b = X_b V V^H: one wave per patch, lanes over the pixels (chunks of 64);
// the patch's r Q entries of V are read once into LDS and broadcast from there
__global__ void __launch_bounds__(64) k_llr_project(const float2* __restrict__ X,
                                                    const float2* __restrict__ V,
                                                    float2* __restrict__ Xr, long long B, int Q,
                                                    int m, int r) {
  __shared__ float2 vs[8 * kMaxQ];
  const long long b = xcd_block(blockIdx.x, gridDim.x);
  if (b >= B) return;
  const int l = threadIdx.x;
  for (int e = l; e < r * Q; e += 64) vs[e] = V[size_t(e) * B + b];
  __syncthreads();
  const float2* xb = X + size_t(b) * Q * m;
  float2* ob = Xr + size_t(b) * Q * m;
  for (int i = l; i < m; i += 64) {
    float2 c[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) c[k] = make_float2(0.f, 0.f);
    for (int p = 0; p < Q; ++p) {
      const float2 x = xb[size_t(p) * m + i];
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        if (k >= r) break;
        c[k] = cadd(c[k], cmul(x, vs[k * Q + p]));
      }
    }
    for (int q = 0; q < Q; ++q) {
      float2 o = make_float2(0.f, 0.f);
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        if (k >= r) break;
        o = cadd(o, cmul(c[k], cconj(vs[k * Q + q])));
      }
      ob[size_t(q) * m + i] = o;
    }
  }
}

size_t layout_llr(long long B, int Q, int r, void* ws, float2** A, float2** V, float** lam) {
  Carver c(ws);
  float2* a = c.take<float2>(size_t(Q) * (Q + 1) / 2 * B);
  float2* v = c.take<float2>(size_t(r) * Q * B);
  float* l = c.take<float>(size_t(r) * B);
  if (A) *A = a;
  if (V) *V = v;
  if (lam) *lam = l;
  return c.used + 256;
}

pisco_status_t run_llr(Handle* h, long long B, int m, int Q, int r, const float2* X,
                       float* sigma, float2* Vout, float2* Xr, void* ws) {
  if (B <= 0) return PISCO_OK;
  float2 *A, *V;
  float* lam;
  layout_llr(B, Q, r, ws, &A, &V, &lam);
  if (Vout) V = Vout;
  if (Q > 16)
    PISCO_KERNEL(h, k_llr_gram<2>, dim3(unsigned(B)), dim3(64), 0, X, A, B, Q, m,
                 h->status_dev);
  else
    PISCO_KERNEL(h, k_llr_gram<1>, dim3(unsigned(B)), dim3(64), 0, X, A, B, Q, m,
                 h->status_dev);
  pisco_status_t st = run_lanczos_vm(h, Q, B, -1.f, Q, r, A, V, lam, nullptr);
  if (st) return st;
  PISCO_KERNEL(h, k_llr_sigma, dim3(ceil_div(1LL * r * B, 256)), dim3(256), 0, lam, sigma,
               1LL * r * B);
  if (Xr)
    PISCO_KERNEL(h, k_llr_project, dim3(unsigned(B)), dim3(64), 0, X, V, Xr, B, Q, m, r);
  return PISCO_OK;
}

}  // namespace pisco
