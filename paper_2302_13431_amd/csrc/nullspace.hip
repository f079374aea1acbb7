// Signal/null split of the calibration Gram in FP64 (Sec. III-A/B, Eq. 20).
//
// The paper takes the SVD of C and keeps as filters h_r the right singular
// vectors with sigma_n < 0.05 sigma_1.  Because only a few percent of the
// spectrum lies above that level for calibration data, the complement (the
// signal eigenvectors, lambda_n >= 0.05^2 lambda_1 of C^H C) is computed
// instead and the nullspace projector is I - V_s V_s^H, which is the ESPIRiT
// form of Eq. (20).
//
// Method: block subspace iteration with Rayleigh-Ritz on a block of b >= r_s
// columns, all in FP64 on the GPU:
//   Z = A X                        (A = FP32 Gram widened exactly to FP64)
//   X <- orth(Z) by Cholesky QR with column scaling; after the third product
//        up to three products share one orthonormalisation, the scaled
//        block staying well conditioned;
// and, when the rate predicted from the Cholesky diagonal (about the
// eigenvalues in orthogonal iteration) says the block has converged, a
// Rayleigh-Ritz step
//   H = X^H Z, eig(H) = U diag(theta) U^H     (tridiagonal route, heev.hip)
//   W = X U (Ritz vectors), residual_k = ||Z U_k - theta_k W_k||
// that stops the iteration once every Ritz pair up to the first one below
// the threshold has a residual below 1e-10 theta_1 (otherwise the Ritz
// values predict how many more products to run).  The rate per product is
// lambda_{b+1} / lambda_{r_s}, small because the spectrum falls steeply past
// the threshold.
#include <cmath>
#include <utility>

#include "common.hpp"

namespace pisco {

// ------------------------------------------------------------------ init

__device__ inline uint64_t mix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ void k_init_block(double2* X, int n, int b) {
  const long long idx = blockIdx.x * 256LL + threadIdx.x;
  if (idx >= 1LL * n * b) return;
  const uint64_t h = mix64(uint64_t(idx) * 2654435761ull + 12345u);
  const double re = double(h >> 11) * (1.0 / 9007199254740992.0) - 0.5;
  const double im = double(mix64(h) >> 11) * (1.0 / 9007199254740992.0) - 0.5;
  X[idx] = make_double2(re, im);
}

// ------------------------------------------------------------------ GEMMs

// Z_part[ks] = A[:, kslice] X[kslice, :], A float2 row-major n x n (widened to
// FP64), X and Z column-major n x b (double2).  32 x 32 output tile per block,
// 2 x 2 complex micro-tile per thread, K in steps of 32 staged in LDS.
__global__ void __launch_bounds__(256) k_gemm_ax(const float2* __restrict__ A,
                                                 const double2* __restrict__ X,
                                                 double2* __restrict__ Zp, int n, int b,
                                                 int kchunk) {
  __shared__ double2 As[32][33];
  __shared__ double2 Xs[32][33];
  const int t = threadIdx.x;
  const int tr = t >> 4, tc = t & 15;
  const int row0 = blockIdx.x * 32, col0 = blockIdx.y * 32;
  const int kbeg = blockIdx.z * kchunk;
  const int kend = min(n, kbeg + kchunk);
  double2 acc[2][2];
  for (int a = 0; a < 2; ++a)
    for (int c = 0; c < 2; ++c) acc[a][c] = make_double2(0.0, 0.0);
  for (int k0 = kbeg; k0 < kend; k0 += 32) {
    for (int e = t; e < 1024; e += 256) {
      const int rr = e >> 5, kk = e & 31;
      const int gr = row0 + rr, gk = k0 + kk;
      double2 v = make_double2(0.0, 0.0);
      if (gr < n && gk < kend) {
        const float2 f = A[size_t(gr) * n + gk];
        v = make_double2(double(f.x), double(f.y));
      }
      As[rr][kk] = v;
      const int cc = e >> 5;  // column of X
      const int gc = col0 + cc;
      double2 x = make_double2(0.0, 0.0);
      if (gc < b && gk < kend) x = X[size_t(gc) * n + gk];
      Xs[kk][cc] = x;
    }
    __syncthreads();
#pragma unroll 8
    for (int kk = 0; kk < 32; ++kk) {
      const double2 a0 = As[tr * 2][kk], a1 = As[tr * 2 + 1][kk];
      const double2 x0 = Xs[kk][tc * 2], x1 = Xs[kk][tc * 2 + 1];
      acc[0][0] = zadd(acc[0][0], zmul(a0, x0));
      acc[0][1] = zadd(acc[0][1], zmul(a0, x1));
      acc[1][0] = zadd(acc[1][0], zmul(a1, x0));
      acc[1][1] = zadd(acc[1][1], zmul(a1, x1));
    }
    __syncthreads();
  }
  double2* out = Zp + size_t(blockIdx.z) * n * b;
  for (int a = 0; a < 2; ++a)
    for (int c = 0; c < 2; ++c) {
      const int gr = row0 + tr * 2 + a, gc = col0 + tc * 2 + c;
      if (gr < n && gc < b) out[size_t(gc) * n + gr] = acc[a][c];
    }
}

// out = sum over `parts` slabs of size `len` (fixed order: deterministic)
__global__ void k_sum_parts(const double2* __restrict__ parts, double2* __restrict__ out,
                            long long len, int nparts) {
  const long long i = blockIdx.x * 256LL + threadIdx.x;
  if (i >= len) return;
  double2 s = parts[i];
  for (int k = 1; k < nparts; ++k) s = zadd(s, parts[size_t(k) * len + i]);
  out[i] = s;
}

// part[chunk] = P[rows of chunk, :]^H Q[rows of chunk, :]; P, Q column-major
// n x b; part is column-major b x b.  Rows are split in chunks of 256.
__global__ void __launch_bounds__(256) k_gemm_tn(const double2* __restrict__ P,
                                                 const double2* __restrict__ Qm,
                                                 double2* __restrict__ part, int n, int b) {
  __shared__ double2 Ps[32][33];
  __shared__ double2 Qs[32][33];
  const int t = threadIdx.x;
  const int ti = t >> 4, tj = t & 15;
  const int i0 = blockIdx.x * 32, j0 = blockIdx.y * 32;
  const int rbeg = blockIdx.z * 256, rend = min(n, rbeg + 256);
  double2 acc[2][2];
  for (int a = 0; a < 2; ++a)
    for (int c = 0; c < 2; ++c) acc[a][c] = make_double2(0.0, 0.0);
  for (int r0 = rbeg; r0 < rend; r0 += 32) {
    for (int e = t; e < 1024; e += 256) {
      const int cc = e >> 5, rr = e & 31;
      const int gr = r0 + rr;
      double2 pv = make_double2(0.0, 0.0), qv = make_double2(0.0, 0.0);
      if (gr < rend) {
        if (i0 + cc < b) pv = P[size_t(i0 + cc) * n + gr];
        if (j0 + cc < b) qv = Qm[size_t(j0 + cc) * n + gr];
      }
      Ps[rr][cc] = pv;
      Qs[rr][cc] = qv;
    }
    __syncthreads();
#pragma unroll 8
    for (int rr = 0; rr < 32; ++rr) {
      const double2 p0 = Ps[rr][ti * 2], p1 = Ps[rr][ti * 2 + 1];
      const double2 q0 = Qs[rr][tj * 2], q1 = Qs[rr][tj * 2 + 1];
      acc[0][0] = zadd(acc[0][0], zmulc(p0, q0));
      acc[0][1] = zadd(acc[0][1], zmulc(p0, q1));
      acc[1][0] = zadd(acc[1][0], zmulc(p1, q0));
      acc[1][1] = zadd(acc[1][1], zmulc(p1, q1));
    }
    __syncthreads();
  }
  double2* out = part + size_t(blockIdx.z) * b * b;
  for (int a = 0; a < 2; ++a)
    for (int c = 0; c < 2; ++c) {
      const int gi = i0 + ti * 2 + a, gj = j0 + tj * 2 + c;
      if (gi < b && gj < b) out[size_t(gj) * b + gi] = acc[a][c];
    }
}

// Y = P M; P column-major m x k, M column-major k x b, Y column-major m x b.
__global__ void __launch_bounds__(256) k_gemm_nn(const double2* __restrict__ Pm,
                                                 const double2* __restrict__ M,
                                                 double2* __restrict__ Y, int m, int k,
                                                 int b) {
  __shared__ double2 Ps[32][33];
  __shared__ double2 Ms[32][33];
  const int t = threadIdx.x;
  const int tr = t >> 4, tc = t & 15;
  const int r0 = blockIdx.x * 32, c0 = blockIdx.y * 32;
  double2 acc[2][2];
  for (int a = 0; a < 2; ++a)
    for (int c = 0; c < 2; ++c) acc[a][c] = make_double2(0.0, 0.0);
  for (int k0 = 0; k0 < k; k0 += 32) {
    for (int e = t; e < 1024; e += 256) {
      const int cc = e >> 5, rr = e & 31;
      double2 pv = make_double2(0.0, 0.0), mv = make_double2(0.0, 0.0);
      if (r0 + rr < m && k0 + cc < k) pv = Pm[size_t(k0 + cc) * m + r0 + rr];
      if (k0 + rr < k && c0 + cc < b) mv = M[size_t(c0 + cc) * k + k0 + rr];
      Ps[rr][cc] = pv;   // [row][kk]
      Ms[rr][cc] = mv;   // [kk][col]
    }
    __syncthreads();
#pragma unroll 8
    for (int kk = 0; kk < 32; ++kk) {
      const double2 p0 = Ps[tr * 2][kk], p1 = Ps[tr * 2 + 1][kk];
      const double2 m0 = Ms[kk][tc * 2], m1 = Ms[kk][tc * 2 + 1];
      acc[0][0] = zadd(acc[0][0], zmul(p0, m0));
      acc[0][1] = zadd(acc[0][1], zmul(p0, m1));
      acc[1][0] = zadd(acc[1][0], zmul(p1, m0));
      acc[1][1] = zadd(acc[1][1], zmul(p1, m1));
    }
    __syncthreads();
  }
  for (int a = 0; a < 2; ++a)
    for (int c = 0; c < 2; ++c) {
      const int gr = r0 + tr * 2 + a, gc = c0 + tc * 2 + c;
      if (gr < m && gc < b) Y[size_t(gc) * m + gr] = acc[a][c];
    }
}

// ------------------------------------------------------------------ Cholesky QR

constexpr int kCholLdsMax = 96;  // largest b factored with the matrix in LDS

// Cholesky factor of D S D + shift I, so that Y M has orthonormal columns
// when S = Y^H Y (up to the shift).  One block; the working matrix is in LDS
// when kLds (b <= 96) and in `gwork` otherwise.  A pivot that is not positive
// is replaced by a tiny one and reported through *flag.
template <bool kLds>
__global__ void __launch_bounds__(1024) k_chol_inv(const double2* __restrict__ S, int b,
                                                   double shift, double2* __restrict__ M,
                                                   double2* __restrict__ gwork,
                                                   int* __restrict__ flag,
                                                   double* __restrict__ rdiag) {
  // T is row-major with a padded leading dimension ld = b + 1, so that rows
  // are contiguous for the factorisation and the column walks of the inverse
  // spread over the LDS banks
  __shared__ double2 lds_mat[kLds ? kCholLdsMax * (kCholLdsMax + 1) : 1];
  __shared__ double dsc[kLds ? kCholLdsMax : 1024];
  double2* T = kLds ? lds_mat : gwork;
  const int ld = b + 1;
  const int t = threadIdx.x, nt = blockDim.x;
  for (int k = t; k < b; k += nt) {
    const double d = S[size_t(k) * b + k].x;
    dsc[k] = d > 0.0 ? 1.0 / sqrt(d) : 0.0;
  }
  __syncthreads();
  for (int e = t; e < b * b; e += nt) {
    const int i = e % b, j = e / b;  // S is column-major: e = j b + i
    double2 v = zscale(S[e], dsc[i] * dsc[j]);
    if (i == j) v = make_double2(v.x + shift, 0.0);
    T[size_t(i) * ld + j] = v;
  }
  __syncthreads();
  // blocked right-looking Cholesky on the upper triangle, T = R^H R, with
  // panels of kPW columns: (a) the first wave factors the diagonal block
  // (wave-level ordering only), (b) each remaining column solves the panel's
  // triangular system, (c) all threads apply the rank-kPW trailing update.
  constexpr int kPW = 16;
  __shared__ double dinv[kPW];
  for (int k0 = 0; k0 < b; k0 += kPW) {
    const int k1 = k0 + kPW < b ? k0 + kPW : b;
    if (t < 64) {
      for (int k = k0; k < k1; ++k) {
        double2* rk = T + size_t(k) * ld;
        double dk = rk[k].x;
        if (!(dk > 1e-300)) {
          if (t == 0) *flag = 1;
          dk = 1e-300;
        }
        const double r = sqrt(dk), rinv = 1.0 / r;
        // diagonal of the unscaled factor (R' D^-1): converges to the
        // eigenvalue magnitudes in orthogonal iteration
        if (rdiag && t == 0) rdiag[k] = dsc[k] > 0.0 ? r / dsc[k] : 0.0;
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        if (t < k1 - k) rk[k + t] = t == 0 ? make_double2(r, 0.0) : zscale(rk[k + t], rinv);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        // update the rest of the diagonal block: rows i in (k, k1), j >= i
        const int m = k1 - k - 1;
        for (int e = t; e < m * m; e += 64) {
          const int i = k + 1 + e / m, j = k + 1 + e % m;
          if (j >= i)
            T[size_t(i) * ld + j] = zsub(T[size_t(i) * ld + j], zmulc(rk[i], rk[j]));
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
      }
    }
    __syncthreads();
    for (int k = k0 + t; k < k1; k += nt) dinv[k - k0] = 1.0 / T[size_t(k) * ld + k].x;
    __syncthreads();
    // (b) R_{k0:k1, j} = R_pp^{-H} T_{k0:k1, j} for every column j >= k1
    for (int j = k1 + t; j < b; j += nt) {
      for (int k = k0; k < k1; ++k) {
        double2 acc = T[size_t(k) * ld + j];
        for (int l = k0; l < k; ++l)
          acc = zsub(acc, zmulc(T[size_t(l) * ld + k], T[size_t(l) * ld + j]));
        T[size_t(k) * ld + j] = zscale(acc, dinv[k - k0]);
      }
    }
    __syncthreads();
    // (c) T_{i,j} -= sum_{l in panel} conj(R_{l,i}) R_{l,j},  k1 <= i <= j
    const int m = b - k1;
    for (int e = t; e < m * m; e += nt) {
      const int i = k1 + e / m, j = k1 + e % m;
      if (j < i) continue;
      double2 acc = T[size_t(i) * ld + j];
      for (int l = k0; l < k1; ++l)
        acc = zsub(acc, zmulc(T[size_t(l) * ld + i], T[size_t(l) * ld + j]));
      T[size_t(i) * ld + j] = acc;
    }
    __syncthreads();
  }
  if (kLds) {
    // M(:, j) = D R^{-1} e_j by back substitution, one group of 8 lanes per
    // column j; entry l of the column lives in register slot l / 8 of lane
    // l % 8 and each step's dot product is a butterfly over the group.
    constexpr int G = 8, SL = kCholLdsMax / G;
    __shared__ double rinv[kCholLdsMax];
    for (int i = t; i < b; i += nt) rinv[i] = 1.0 / T[size_t(i) * ld + i].x;
    __syncthreads();
    // column j of R^{-1} by a column-oriented back substitution: start from
    // e_j, and for i = j, j-1, ..., 0 scale entry i by 1/R_ii, broadcast it
    // to the group and subtract its multiple of column i of R from the
    // entries above it.  No reductions; one broadcast per step.
    const int j = t / G, lane = t % G;
    double2 mreg[SL];
#pragma unroll
    for (int k = 0; k < SL; ++k) {
      const int l = lane + k * G;
      mreg[k] = make_double2(l == j ? 1.0 : 0.0, 0.0);
    }
    if (j < b) {
      for (int i = j; i >= 0; --i) {
        // owner of entry i scales it; everyone reads it
        double2 mi = make_double2(0.0, 0.0);
#pragma unroll
        for (int k = 0; k < SL; ++k)
          if (k == i / G) mi = mreg[k];
        mi = zscale(mi, rinv[i]);
        const int src = (t & ~(G - 1)) + (i % G);
        mi.x = __shfl(mi.x, src, 64);
        mi.y = __shfl(mi.y, src, 64);
#pragma unroll
        for (int k = 0; k < SL; ++k) {
          const int l = lane + k * G;
          if (l == i) mreg[k] = mi;
          else if (l < i) mreg[k] = zsub(mreg[k], zmul(T[size_t(l) * ld + i], mi));
        }
      }
#pragma unroll
      for (int k = 0; k < SL; ++k) {
        const int l = lane + k * G;
        if (l < b)
          M[size_t(j) * b + l] = l <= j ? zscale(mreg[k], dsc[l]) : make_double2(0.0, 0.0);
      }
    }
    return;
  }
  // global-memory variant: in-place inverse of the upper triangle, column by
  // column (with the leading j x j block already inverted, column j of R^{-1}
  // is -(R^{-1})_{0:j,0:j} R_{0:j,j} / R_jj, and 1 / R_jj on the diagonal)
  __shared__ double2 xcol[kLds ? 1 : 1024];
  for (int j = 0; j < b; ++j) {
    for (int i = t; i < j; i += nt) xcol[i] = T[size_t(i) * ld + j];
    __syncthreads();
    const double inv_jj = 1.0 / T[size_t(j) * ld + j].x;
    for (int i = t; i < j; i += nt) {
      double2 acc = make_double2(0.0, 0.0);
      for (int l = i; l < j; ++l) acc = zadd(acc, zmul(T[size_t(i) * ld + l], xcol[l]));
      T[size_t(i) * ld + j] = zscale(acc, -inv_jj);
    }
    __syncthreads();
    if (t == 0) T[size_t(j) * ld + j] = make_double2(inv_jj, 0.0);
  }
  __syncthreads();
  // M = D R^{-1} (rows scaled), column-major, zero below the diagonal
  for (int e = t; e < b * b; e += nt) {
    const int i = e % b, j = e / b;
    M[e] = i <= j ? zscale(T[size_t(i) * ld + j], dsc[i]) : make_double2(0.0, 0.0);
  }
}

// part[chunk][k] = sum over rows of chunk of |Y_k - theta_k W_k|^2
__global__ void __launch_bounds__(256) k_colresid(const double2* __restrict__ Y,
                                                  const double2* __restrict__ W,
                                                  const double* __restrict__ theta,
                                                  double* __restrict__ part, int n, int b) {
  __shared__ double red[256];
  const int k = blockIdx.y;
  const int rbeg = blockIdx.x * 1024;
  const double th = theta[k];
  double s = 0.0;
  for (int r = rbeg + threadIdx.x; r < min(n, rbeg + 1024); r += 256) {
    const double2 y = Y[size_t(k) * n + r], w = W[size_t(k) * n + r];
    s += zabs2(make_double2(y.x - th * w.x, y.y - th * w.y));
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[size_t(blockIdx.x) * b + k] = red[0];
}

// Control: count signal Ritz values, test convergence, predict.
//   ctl[0] = r_signal, ctl[1] = converged, ctl[2] = iterations,
//   ctl[3] = block too small, ctl[4] = all-zero data,
//   ctl[5] = plain steps predicted before the next Rayleigh-Ritz
__global__ void k_control(const double* __restrict__ theta, const double* __restrict__ rpart,
                          int nchunks, int b, double thr2, double tol, int margin, int iter,
                          int* ctl, unsigned* status) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double t0 = theta[0];
  int rs = 0;
  for (int k = 0; k < b; ++k) rs += theta[k] >= thr2 * t0;
  const int upto = rs + 1 < b ? rs + 1 : b;
  double worst = 0.0;
  bool finite = isfinite(t0);
  for (int k = 0; k < upto; ++k) {
    double s = 0.0;
    for (int c = 0; c < nchunks; ++c) s += rpart[size_t(c) * b + k];
    const double r = sqrt(s);
    if (!isfinite(r)) finite = false;
    worst = r > worst ? r : worst;
  }
  const int zero = !(t0 > 0.0);
  if (zero) rs = 0;
  const int too_small = rs > b - margin;
  ctl[0] = rs;
  ctl[1] = (finite && !zero && worst <= tol * t0 && !too_small) ? 1 : 0;
  ctl[2] = iter + 1;
  ctl[3] = too_small;
  ctl[4] = zero;
  // iterations predicted to reach the tolerance at rate theta_b / theta_rs
  int need = 1;
  if (rs > 0 && worst > tol * t0 && finite && !zero) {
    double rho = theta[b - 1] / theta[rs - 1];
    rho = rho < 1e-3 ? 1e-3 : (rho > 0.95 ? 0.95 : rho);
    const double k = log(tol * t0 / worst) / log(rho);
    need = int(ceil(k)) + 1;
    need = need < 1 ? 1 : (need > 20 ? 20 : need);
  }
  ctl[5] = need;
  if (!finite) atomicOr(status, PISCO_FLAG_NONFINITE);
}

// Iterations still needed, predicted from the Cholesky diagonal d_j (about
// lambda_j): rate d_{b-1} / d_{r}, r the number of d_j >= thr2 d_0, from an
// error of order one after `done` products.  ctl[6] = prediction.
__global__ void k_predict(const double* __restrict__ d, int b, double thr2, double tol,
                          int done, int* ctl) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int r = 0;
  for (int k = 0; k < b; ++k) r += d[k] >= thr2 * d[0];
  int need = 4;
  if (r > 0 && r < b && d[r - 1] > 0.0) {
    double rho = d[b - 1] / d[r - 1];
    rho = rho < 1e-3 ? 1e-3 : (rho > 0.95 ? 0.95 : rho);
    need = int(ceil(log(tol) / log(rho))) - done + 1;
  }
  ctl[6] = need < 1 ? 1 : (need > 40 ? 40 : need);
}

__global__ void k_finalize(const double2* __restrict__ W, const double* __restrict__ theta,
                           const int* __restrict__ ctl, double2* __restrict__ basis,
                           double* __restrict__ eigvals, int32_t* __restrict__ counts,
                           long long nb, int b, unsigned* status) {
  const long long i = blockIdx.x * 256LL + threadIdx.x;
  if (i < nb) basis[i] = W[i];
  if (i < b) eigvals[i] = theta[i];
  if (i == 0) {
    counts[0] = ctl[0];
    counts[1] = b;
    counts[2] = ctl[2];
    counts[3] = ctl[1];
    unsigned f = 0;
    if (!ctl[1]) f |= PISCO_FLAG_NOT_CONVERGED;
    if (ctl[3]) f |= PISCO_FLAG_BLOCK_TOO_SMALL;
    if (ctl[4]) f |= PISCO_FLAG_ZERO_DATA;
    if (f) atomicOr(status, f);
  }
}

// ------------------------------------------------------------------ driver

namespace {

struct NullCtx {
  Handle* h;
  const Plan* p;
  int b;
  NullWs w;
};

pisco_status_t gemm_tn(NullCtx& c, const double2* P, const double2* Qm, double2* out, int rows) {
  const int b = c.b;
  const int chunks = int(ceil_div(rows, 256));
  dim3 g(ceil_div(b, 32), ceil_div(b, 32), chunks);
  PISCO_KERNEL(c.h, k_gemm_tn, g, dim3(256), 0, P, Qm, c.w.part, rows, b);
  const long long len = 1LL * b * b;
  PISCO_KERNEL(c.h, k_sum_parts, dim3(ceil_div(len, 256)), dim3(256), 0, c.w.part, out, len, chunks);
  return PISCO_OK;
}

pisco_status_t gemm_nn(NullCtx& c, const double2* P, const double2* M, double2* Y, int m,
                       int k) {
  dim3 g(ceil_div(m, 32), ceil_div(c.b, 32));
  PISCO_KERNEL(c.h, k_gemm_nn, g, dim3(256), 0, P, M, Y, m, k, c.b);
  return PISCO_OK;
}

pisco_status_t chol_inv(NullCtx& c, const double2* S, double shift, double2* M,
                        double* rdiag = nullptr) {
  const int b = c.b;
  int* flag = c.w.ctl + 8;
  if (b <= kCholLdsMax)
    PISCO_KERNEL(c.h, k_chol_inv<true>, dim3(1), dim3(1024), 0, S, b, shift, M,
                 reinterpret_cast<double2*>(c.w.jac), flag, rdiag);
  else
    PISCO_KERNEL(c.h, k_chol_inv<false>, dim3(1), dim3(1024), 0, S, b, shift, M,
                 reinterpret_cast<double2*>(c.w.jac), flag, rdiag);
  return PISCO_OK;
}

// Orthonormalise the columns of Y (n x b) by Cholesky QR with column scaling
// (the first pass with a tiny diagonal shift against breakdown).  Two passes
// (result back in Y, `tmp` is scratch) while the columns may be nearly
// dependent; one pass (result in `tmp`) once they are close to orthogonal
// after scaling, where a single pass is already accurate to rounding.
pisco_status_t orth(NullCtx& c, double2* Y, double2* tmp, double* rdiag = nullptr,
                    int passes = 2) {
  const int n = c.p->n, b = c.b;
  pisco_status_t st;
  if ((st = gemm_tn(c, Y, Y, c.w.S, n))) return st;
  if ((st = chol_inv(c, c.w.S, passes == 2 ? 1e-12 : 0.0, c.w.M, rdiag))) return st;
  if ((st = gemm_nn(c, Y, c.w.M, tmp, n, b))) return st;
  if (passes == 1) return PISCO_OK;
  if ((st = gemm_tn(c, tmp, tmp, c.w.S, n))) return st;
  if ((st = chol_inv(c, c.w.S, 0.0, c.w.M))) return st;
  return gemm_nn(c, tmp, c.w.M, Y, n, b);
}

}  // namespace

pisco_status_t run_nullspace(Handle* h, const Plan& p, int b, int max_iters,
                             const float2* gram, double* eigvals, double2* basis,
                             int32_t* counts, void* ws) {
  NullCtx c{h, &p, b, {}};
  layout_null(p, b, ws, &c.w);
  hipStream_t s = h->stream;
  const int n = p.n;
  const long long nb = 1LL * n * b;
  double2* W = basis;  // Ritz vectors are formed directly in the output buffer
  double2* X = c.w.X;  // current orthonormal block
  double2* Z = c.w.Z;  // A X

  PISCO_KERNEL(h, k_init_block, dim3(ceil_div(nb, 256)), dim3(256), 0, X, n, b);
  // a random block is well conditioned: one Cholesky QR pass
  pisco_status_t st = orth(c, X, Z, nullptr, 1);
  if (st) return st;
  std::swap(X, Z);

  const double thr2 = double(p.thresh) * double(p.thresh);
  const double tol = 1e-10;
  const int margin = b / 8 > 4 ? b / 8 : 4;
  const int kchunk = 256 * int(ceil_div(ceil_div(n, 4), 256));
  const int ksplit = int(ceil_div(n, kchunk));
  const int rchunks = int(ceil_div(n, 1024));
  // Z = A X (split-K partials in `part`, summed in fixed order)
  auto product = [&](const double2* in, double2* out) -> pisco_status_t {
    dim3 g(ceil_div(n, 32), ceil_div(b, 32), ksplit);
    PISCO_KERNEL(h, k_gemm_ax, g, dim3(256), 0, gram, in, c.w.part, n, b, kchunk);
    PISCO_KERNEL(h, k_sum_parts, dim3(ceil_div(nb, 256)), dim3(256), 0, c.w.part, out, nb,
                 ksplit);
    return PISCO_OK;
  };
  // Products are counted in `done`.  The first Rayleigh-Ritz step is
  // scheduled from the Cholesky diagonal seen after three products, later
  // ones from the Ritz values and residuals.  After the third product the
  // scaled block stays well conditioned (kappa of order 10 for two more
  // products), so up to three products share one Cholesky QR pass.
  constexpr int kUnscheduled = 1 << 30;
  int rr_at = kUnscheduled;  // product count at which to run Rayleigh-Ritz
  int done = 0;
  while (true) {
    if ((st = product(X, Z))) return st;
    ++done;
    if (done < rr_at && done < max_iters) {
      int extra = 0;
      if (done >= 3 && rr_at != kUnscheduled) {
        extra = rr_at - done - 1;
        extra = extra < 0 ? 0 : (extra > 2 ? 2 : extra);
      }
      for (int e = 0; e < extra; ++e) {
        if ((st = product(Z, X))) return st;
        std::swap(X, Z);
        ++done;
      }
      const bool predict = done == 3 && rr_at == kUnscheduled;
      const int passes = done == 1 ? 2 : 1;
      if ((st = orth(c, Z, X, predict ? c.w.resid : nullptr, passes))) return st;
      if (passes == 2) std::swap(X, Z);  // two passes leave the result in Z
      if (predict) {
        PISCO_KERNEL(h, k_predict, dim3(1), dim3(64), 0, c.w.resid, b, thr2, tol, done,
                     c.w.ctl);
        hipError_t e = hipMemcpyAsync(h->host_pinned, c.w.ctl, 8 * sizeof(int),
                                      hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_check(h, e, "nullspace predict");
        rr_at = done + reinterpret_cast<const int*>(h->host_pinned)[6];
      }
      continue;
    }
    // Rayleigh-Ritz on span(X): H = X^H A X = U diag(theta) U^H
    if ((st = gemm_tn(c, X, Z, c.w.H, n))) return st;
    if ((st = run_heev(h, c.w.H, b, c.w.U, c.w.theta, c.w.heev))) return st;
    if ((st = gemm_nn(c, X, c.w.U, W, n, b))) return st;  // Ritz vectors
    if ((st = gemm_nn(c, Z, c.w.U, X, n, b))) return st;  // A * Ritz vectors
    double* rpart = reinterpret_cast<double*>(c.w.part);
    PISCO_KERNEL(h, k_colresid, dim3(rchunks, b), dim3(256), 0, X, W, c.w.theta, rpart, n, b);
    PISCO_KERNEL(h, k_control, dim3(1), dim3(64), 0, c.w.theta, rpart, rchunks, b, thr2, tol,
                 margin, done - 1, c.w.ctl, h->status_dev);
    hipError_t e = hipMemcpyAsync(h->host_pinned, c.w.ctl, 6 * sizeof(int),
                                  hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return hip_check(h, e, "nullspace ctl copy");
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_check(h, e, "nullspace sync");
    const int* hc = reinterpret_cast<const int*>(h->host_pinned);
    if (hc[1] || hc[3] || hc[4]) break;
    if (done >= max_iters) break;
    rr_at = done + hc[5];
    // next block: orth(A * Ritz vectors) (held in X; nearly orthogonal columns)
    if ((st = orth(c, X, Z, nullptr, 1))) return st;
    std::swap(X, Z);
  }
  PISCO_KERNEL(h, k_finalize, dim3(ceil_div(nb > b ? nb : b, 256)), dim3(256), 0, W, c.w.theta, c.w.ctl, basis, eigvals, counts, nb, b, h->status_dev);
  return PISCO_OK;
}

}  // namespace pisco
