// Gram products through the correlation structure of the Gram (Sec. IV-A,
// Eqs. 21-22), without forming the Gram.
//
// Gram[(p,i),(q,j)] = R_pq[n_i - n_j] with the lags d = n_i - n_j in
// [-2 tau, 2 tau]^D, so for a block X of b columns
//   (A x)_p(n) = sum_q sum_m R_pq[n - m] x_q(m),    n, m in the support,
// a sum of D-dimensional correlations.  On a frequency grid of F = 4 tau + 1
// points per dimension (the lag window exactly: n - m never aliases) this is
//   Y_p(f) = sum_q Rhat_pq(f) X_q(f),
// with X_q(f) = sum_m x_q(m) e^{-2 pi i f m / F} over the support box
// [-tau, tau]^D and y(n) = F^{-D} sum_f Y(f) e^{+2 pi i f n / F} on the box.
// Rhat(f) is Hermitian per frequency (R_qp[d] = conj(R_pq[-d])); the
// diagonal is taken real, which is the transform of the Hermitian part of
// R_pp, so the operator is exactly Hermitian like the explicit Gram.
//
// One product (FP64): scatter the block onto the box, three pruned DFT
// passes (box -> frequency, the separable one-axis transform), one
// (b x Q)(Q x Q) product per frequency, three passes back (frequency ->
// box), gather the support points with the Chebyshev-step epilogue of the
// explicit product.  The spectra are laid out frequency-major with the b Q
// block innermost ([f][c][q]), so that every pass reads and writes whole
// contiguous runs and each frequency's block is one contiguous matrix.
// Work per product: 8 F^D Q^2 b flops for the per-frequency products plus
// the passes, against 8 n^2 b for the explicit Gram (n = Q |Lambda|).
#include "common.hpp"

namespace pisco {

namespace {

__device__ inline int tp_pidx(int p, int q, int Q) {  // p <= q
  return p * Q - p * (p - 1) / 2 + (q - p);
}

// rhat[f][p][q] from the transformed lags lf[pair][f]: conj below the
// diagonal, real diagonal
__global__ void k_tp_rhat(const double2* __restrict__ lf, double2* __restrict__ rhat, int Q,
                          long long nf) {
  const long long idx = blockIdx.x * 256LL + threadIdx.x;
  if (idx >= nf * Q * Q) return;
  const long long f = idx / (Q * Q);
  const int e = int(idx - f * Q * Q), p = e / Q, q = e - p * Q;
  const int lo = p < q ? p : q, hi = p < q ? q : p;
  double2 v = lf[size_t(tp_pidx(lo, hi, Q)) * nf + f];
  if (p > q) v.y = -v.y;
  if (p == q) v.y = 0.0;
  rhat[idx] = v;
}

// box[cell][c][q] = X[c][q L + boxmap[cell]], zero off the support
__global__ void k_tp_scatter(const double2* __restrict__ X, const int* __restrict__ boxmap,
                             double2* __restrict__ box, int n, int L, int Q, int b, int cells,
                             const int* __restrict__ role) {
  if (role && *role == 0) return;
  const long long idx = blockIdx.x * 256LL + threadIdx.x;
  if (idx >= 1LL * cells * b * Q) return;
  const int q = int(idx % Q);
  const long long cq = idx / Q;
  const int c = int(cq % b), cell = int(cq / b);
  const int s = boxmap[cell];
  box[idx] = s >= 0 ? X[size_t(c) * n + size_t(q) * L + s] : make_double2(0.0, 0.0);
}

typedef double f64x4 __attribute__((ext_vector_type(4)));

// Yh[f][c][p] = sum_q rhat[f][p][q] Xh[f][c][q] on the FP64 matrix cores:
// per frequency (blockIdx.y) a (b x Q)(Q x Q) product, four waves of 16
// columns c each (blockIdx.x picks 64 columns), both 16-wide tiles of p.
// Complex products in the three-multiplication form (T1 = Xr Rr, T2 = Xi
// Ri, T3 = (Xr + Xi)(Rr + Ri); Re = T1 - T2, Im = T3 - T1 - T2).  Operand
// lanes: lane l supplies row (column) l % 16 at q = 4 s + l / 16 for step
// s; accumulator element v of lane l is c = l / 16 + 4 v, p = l % 16.
__global__ void __launch_bounds__(256) k_tp_pointwise(const double2* __restrict__ Xh,
                                                      const double2* __restrict__ rhat,
                                                      double2* __restrict__ Yh, int Q, int b,
                                                      const int* __restrict__ role) {
  if (role && *role == 0) return;
  const long long f = blockIdx.y;
  const int l = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int li = l & 15, lk = l >> 4;
  const int c0 = blockIdx.x * 64 + wv * 16;
  if (c0 >= b) return;  // the whole wave
  const double2* X = Xh + size_t(f) * b * Q;
  const double2* R = rhat + size_t(f) * Q * Q;
  const bool crow = c0 + li < b;
  f64x4 t1[2], t2[2], t3[2];
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    t1[j] = f64x4{0.0, 0.0, 0.0, 0.0};
    t2[j] = f64x4{0.0, 0.0, 0.0, 0.0};
    t3[j] = f64x4{0.0, 0.0, 0.0, 0.0};
  }
#pragma unroll
  for (int s = 0; s < kMaxQ / 4; ++s) {
    const int q = 4 * s + lk;
    if (4 * s >= Q) break;
    const double2 x = crow && q < Q ? X[size_t(c0 + li) * Q + q] : make_double2(0.0, 0.0);
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int p = 16 * j + li;
      const double2 r = p < Q && q < Q ? R[p * Q + q] : make_double2(0.0, 0.0);
      t1[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(x.x, r.x, t1[j], 0, 0, 0);
      t2[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(x.y, r.y, t2[j], 0, 0, 0);
      t3[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(x.x + x.y, r.x + r.y, t3[j], 0, 0, 0);
    }
  }
  double2* Y = Yh + size_t(f) * b * Q;
#pragma unroll
  for (int j = 0; j < 2; ++j)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int c = c0 + lk + 4 * v, p = 16 * j + li;
      if (c < b && p < Q)
        Y[size_t(c) * Q + p] = make_double2(t1[j][v] - t2[j][v], t3[j][v] - t1[j][v] - t2[j][v]);
    }
}

// out[c][p L + i] from box[cell(i)][c][p]: S, or a S + bc X + g prev with
// (a, bc, g) = coef[0..2] (coef[3..5] for role 2); role 0 copies X
__global__ void k_tp_gather(const double2* __restrict__ box, const int4* __restrict__ sup,
                            const double2* __restrict__ X, double2* out,
                            const double2* prev, int n, int L, int Q, int b, int W, int tz,
                            int tau, const double* __restrict__ coef,
                            const int* __restrict__ role) {
  const long long idx = blockIdx.x * 256LL + threadIdx.x;
  if (idx >= 1LL * b * n) return;
  const int c = int(idx / n), r = int(idx - 1LL * c * n);
  const int p = r / L, i = r - p * L;
  if (role) {
    const int rl = *role;
    if (rl == 0) {
      out[idx] = X[idx];
      return;
    }
    if (rl == 2) coef += 3;
  }
  const int4 s = sup[i];
  const int cell = ((s.x + tz) * W + (s.y + tau)) * W + (s.z + tau);
  const double2 v = box[(size_t(cell) * b + c) * Q + p];
  double2 res = v;
  if (coef) {
    const double2 y = X[idx];
    res = make_double2(coef[0] * v.x + coef[1] * y.x, coef[0] * v.y + coef[1] * y.y);
    if (prev) {
      const double2 q = prev[idx];
      res.x += coef[2] * q.x;
      res.y += coef[2] * q.y;
    }
  }
  out[idx] = res;
}

}  // namespace

size_t toeplitz_spectrum_elems(const Plan& p, int b) {
  return size_t(p.K[0]) * p.K[1] * p.K[2] * size_t(b) * p.Q;
}

pisco_status_t toeplitz_prepare(Handle* h, const ToeplitzOp& op) {
  // lags [P][Bz][B][B] -> [P][Fz][F][F] (FP64), then the per-frequency
  // Hermitian matrices
  const int P = op.P, B = op.F, Bz = op.Fz, F = op.F, Fz = op.Fz;
  pisco_status_t st;
  const int sx[4] = {P * Bz * B, B, 1, 1};
  if ((st = axis_transform64(h, op.lags, op.buf0, sx, 1, F, op.Tr))) return st;
  const int sy[4] = {P * Bz, B, F, 1};
  if ((st = axis_transform64(h, op.buf0, op.buf1, sy, 1, F, op.Tr))) return st;
  const double2* lf = op.buf1;
  if (op.D == 3) {
    const int sz[4] = {P, Bz, F * F, 1};
    if ((st = axis_transform64(h, op.buf1, op.buf0, sz, 1, Fz, op.Tr))) return st;
    lf = op.buf0;
  }
  const long long nf = 1LL * Fz * F * F;
  PISCO_KERNEL(h, k_tp_rhat, dim3(ceil_div(nf * op.Q * op.Q, 256)), dim3(256), 0, lf, op.rhat,
               op.Q, nf);
  return PISCO_OK;
}

pisco_status_t toeplitz_product(Handle* h, const ToeplitzOp& op, const double2* X,
                                double2* out, int n, int b, const double* coef,
                                const double2* prev, const int* role) {
  const int Q = op.Q, W = op.W, Wz = op.Wz, F = op.F, Fz = op.Fz;
  const int bq = b * Q;
  const int cells = Wz * W * W;
  pisco_status_t st;
  PISCO_KERNEL(h, k_tp_scatter, dim3(ceil_div(1LL * cells * bq, 256)), dim3(256), 0, X,
               op.boxmap, op.buf0, n, op.L, Q, b, cells, role);
  // box -> frequency: x, y (, z)
  const int fx[4] = {Wz * W, W, bq, 1};
  if ((st = axis_transform64(h, op.buf0, op.buf1, fx, 1, F, op.Tf))) return st;
  const int fy[4] = {Wz, W, F * bq, 1};
  if ((st = axis_transform64(h, op.buf1, op.buf0, fy, 1, F, op.Tf))) return st;
  double2* spec = op.buf0;
  double2* other = op.buf1;
  if (op.D == 3) {
    const int fz[4] = {1, Wz, F * F * bq, 1};
    if ((st = axis_transform64(h, op.buf0, op.buf1, fz, 1, Fz, op.Tf))) return st;
    spec = op.buf1;
    other = op.buf0;
  }
  const int nf = Fz * F * F;
  PISCO_KERNEL(h, k_tp_pointwise, dim3(ceil_div(b, 64), nf), dim3(256), 0, spec, op.rhat,
               other, Q, b, role);
  // frequency -> box: (z,) y, x
  double2* cur = other;
  double2* nxt = spec;
  if (op.D == 3) {
    const int iz[4] = {1, Fz, F * F * bq, 1};
    if ((st = axis_transform64(h, cur, nxt, iz, 1, Wz, op.Ti))) return st;
    double2* t = cur;
    cur = nxt;
    nxt = t;
  }
  const int iy[4] = {Wz, F, F * bq, 1};
  if ((st = axis_transform64(h, cur, nxt, iy, 1, W, op.Ti))) return st;
  const int ix[4] = {Wz * W, F, bq, 1};
  if ((st = axis_transform64(h, nxt, cur, ix, 1, W, op.Ti))) return st;
  PISCO_KERNEL(h, k_tp_gather, dim3(ceil_div(1LL * b * n, 256)), dim3(256), 0, cur, op.sup, X,
               out, prev, n, op.L, Q, b, W, op.D == 3 ? op.W / 2 : 0, op.W / 2, coef, role);
  return PISCO_OK;
}

}  // namespace pisco
