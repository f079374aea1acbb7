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
#include "common.hpp"

namespace pisco {

// -A_b packed upper, entry-major [Q(Q+1)/2][B]; X is [B][Q][m]
__global__ void k_llr_gram(const float2* __restrict__ X, float2* __restrict__ A, long long B,
                           int Q, int m, unsigned* status) {
  const long long idx = blockIdx.x * 256LL + threadIdx.x;
  const int P = Q * (Q + 1) / 2;
  if (idx >= B * P) return;
  const int pair = int(idx / B);
  const long long b = idx - pair * B;
  int p = 0, base = 0;
  while (pair >= base + (Q - p)) {
    base += Q - p;
    ++p;
  }
  const int q = p + (pair - base);
  const float2* xp = X + (size_t(b) * Q + p) * m;
  const float2* xq = X + (size_t(b) * Q + q) * m;
  float re = 0.f, im = 0.f;
  bool bad = false;
  for (int i = 0; i < m; ++i) {
    const float2 a = xp[i], c = xq[i];
    bad |= !isfinite(a.x) || !isfinite(a.y);
    re = fmaf(a.x, c.x, fmaf(a.y, c.y, re));
    im = fmaf(a.x, c.y, fmaf(-a.y, c.x, im));
  }
  if (bad) atomicOr(status, PISCO_FLAG_NONFINITE);
  A[idx] = p == q ? make_float2(-re, 0.f) : make_float2(-re, -im);
}

// sigma = sqrt(max(lambda(A), 0)) from the eigenvalues of -A
__global__ void k_llr_sigma(const float* __restrict__ lamneg, float* __restrict__ sigma,
                            long long n) {
  const long long i = blockIdx.x * 256LL + threadIdx.x;
  if (i < n) sigma[i] = sqrtf(fmaxf(-lamneg[i], 0.f));
}

// Xr_b = X_b V V^H: one thread per (patch, row)
__global__ void k_llr_project(const float2* __restrict__ X, const float2* __restrict__ V,
                              float2* __restrict__ Xr, long long B, int Q, int m, int r) {
  const long long idx = blockIdx.x * 256LL + threadIdx.x;
  if (idx >= B * m) return;
  const long long b = idx / m;
  const int i = int(idx - b * m);
  float2 c[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) c[k] = make_float2(0.f, 0.f);
  for (int p = 0; p < Q; ++p) {
    const float2 x = X[(size_t(b) * Q + p) * m + i];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      if (k >= r) break;
      const float2 vk = V[(size_t(k) * Q + p) * B + b];
      c[k] = cadd(c[k], cmul(x, vk));
    }
  }
  for (int q = 0; q < Q; ++q) {
    float2 o = make_float2(0.f, 0.f);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      if (k >= r) break;
      o = cadd(o, cmul(c[k], cconj(V[(size_t(k) * Q + q) * B + b])));
    }
    Xr[(size_t(b) * Q + q) * m + i] = o;
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
  const long long P = 1LL * Q * (Q + 1) / 2;
  PISCO_KERNEL(h, k_llr_gram, dim3(ceil_div(B * P, 256)), dim3(256), 0, X, A, B, Q, m,
               h->status_dev);
  pisco_status_t st = run_eig_sets(h, Q, B, -1.f, Q, r, A, V, lam, nullptr);
  if (st) return st;
  PISCO_KERNEL(h, k_llr_sigma, dim3(ceil_div(1LL * r * B, 256)), dim3(256), 0, lam, sigma,
               1LL * r * B);
  if (Xr)
    PISCO_KERNEL(h, k_llr_project, dim3(ceil_div(B * m, 256)), dim3(256), 0, X, V, Xr, B, Q, m,
                 r);
  return PISCO_OK;
}

}  // namespace pisco
