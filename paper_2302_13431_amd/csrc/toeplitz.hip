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
// One product (FP64): the block onto the box and through the x transform
// (one kernel), the y (and z) transforms, one (b x Q)(Q x Q) product per
// frequency (in 3D fused with the z transforms), the inverse y transform,
// and the inverse x transform with the gather of the support points and the
// Chebyshev-step epilogue of the explicit product (one kernel).  The spectra are laid out frequency-major with the b Q
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

// rhat[f][p][q] (rows of kMaxQ, zero past Q, and a zero matrix at f = nf)
// from the transformed lags lf[pair][f]: conj below the diagonal, real
// diagonal
constexpr int kRQ = kMaxQ * kMaxQ;  // elements per frequency
__global__ void k_tp_rhat(const double2* __restrict__ lf, double2* __restrict__ rhat, int Q,
                          long long nf) {
  const long long idx = blockIdx.x * 256LL + threadIdx.x;
  if (idx >= (nf + 1) * kRQ) return;
  const long long f = idx / kRQ;
  const int e = int(idx - f * kRQ), p = e / kMaxQ, q = e - p * kMaxQ;
  double2 v = make_double2(0.0, 0.0);
  if (f < nf && p < Q && q < Q) {
    const int lo = p < q ? p : q, hi = p < q ? q : p;
    v = lf[size_t(tp_pidx(lo, hi, Q)) * nf + f];
    if (p > q) v.y = -v.y;
    if (p == q) v.y = 0.0;
  }
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
  const double2* R = rhat + size_t(f) * kRQ;
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
      const double2 r = R[p * kMaxQ + q];
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

// 3D products: the z pass, the per-frequency products and the inverse z pass
// in one kernel, so that the full spectrum [F^3][b][Q] never reaches memory.
// in  = [Wz][F F][b][Q] after the x and y passes, out = the same layout
// after the inverse z pass; rhat frequency f = (fz F + fy) F + fx.
//
// The z box is centred (z = tau + d, |d| <= tau), so the z transforms pair
// the frequencies f and F - f: with u_d = x(tau + d) + x(tau - d) (u_0 =
// x(tau)), v_d = x(tau + d) - x(tau - d), and Tf[f][tau + d] = cos + i sin,
//   X_f = C + i S,  X_(F-f) = C - i S,  C = sum_d cos_d u_d,  S = sum_d sin_d v_d,
// and back, with S' = Y_f + Y_(F-f), D' = Y_f - Y_(F-f), Ti[tau + d][f] =
// c' + i s' (the 1/F included),
//   out(tau +- d) += c'_d S' +- i s'_d D'
// (a quarter of the multiply-adds of the plain transforms).  The FP64 matrix
// cores and the FP64 vector ALUs do not work at once, so this matters as
// much as the MFMAs.
//
// Tile = one (fy, fx) pair x 16 columns c.  A workgroup walks every G-th
// tile (G workgroups, one per CU; the tiles one XCD holds at a time are
// consecutive, so the tiles of one pair share its matrices in one L2), with
// eight waves
// in two roles (one of each per SIMD); per tile the steps k = 0 .. 2 tau
// take frequency 0 alone, then the pairs (k, F - k); one barrier per step:
//   matrix waves (j, par), w < 4: output channels p in [16 j, 16 j + 16) of
//     the step's frequency par, 24 FP64 MFMAs (three-multiplication complex
//     products, as in k_tp_pointwise), Y into LDS (yb); the matrices of
//     step k + 1 load during step k; and z-plane k of the next tile's input
//     goes into LDS (xn), so that the next tile starts without a wait on
//     HBM;
//   vector waves v = w - 4: X of both frequencies of step k + 1 at the MFMA
//     steps s = 2v, 2v + 1 (u, v of their inputs held in registers) into LDS
//     (xf), and two of the eight output elements per lane accumulated from
//     step k - 1, stored at the end of the tile.
template <int kW>
__global__ void __launch_bounds__(512) k_tp_zfused(const double2* __restrict__ in,
                                                   const double2* __restrict__ rhat,
                                                   const double2* __restrict__ Tf,
                                                   const double2* __restrict__ Ti,
                                                   double2* __restrict__ out, int Q, int b, int F,
                                                   int ctiles, int tiles,
                                                   const int* __restrict__ role) {
  constexpr int kT = kW / 2;     // tau
  constexpr int kS = kMaxQ / 4;  // MFMA steps
  constexpr int QS = kMaxQ + 1;  // padded LDS row of the next tile's input
  static_assert(kS == 8, "two MFMA steps per vector wave");
  __shared__ double2 xf[2][2][kS][64];    // [buffer][frequency of the step][s][lane]
  __shared__ double2 yb[2][2][2][4][64];  // [buffer][frequency of the step][j][v][lane]
  __shared__ double2 xn[kW * 16 * QS];    // the next tile's input [z][c][q]
  if (role && *role == 0) return;
  const int l = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int li = l & 15, lk = l >> 4;
  // this workgroup's tiles: rank, rank + G, ...; the ranks are dealt to the
  // XCDs in contiguous ranges, so that at any time the workgroups of one XCD
  // hold consecutive tiles, which share their pair's matrices in its L2
  const long long G = gridDim.x;
  const long long t0 = xcd_block(blockIdx.x, gridDim.x);
  const size_t FF = size_t(F) * F;
  const size_t zstride = FF * b * Q;
  const int iters = 2 * kT + 1;
  if (w < 4) {
    // matrix waves; the loads of the matrices go without conditions (the
    // zero matrix at FF F when a step has no such frequency), so that the
    // wait before the MFMAs can leave the next step's loads in flight
    const int j = w & 1, par = w >> 1;
    const int p = 16 * j + li;
    const int tl = threadIdx.x;  // 0 .. 255 over the matrix waves
    for (long long tile = t0; tile < tiles; tile += G) {
      const int pair = int(tile / ctiles);
      const bool more = tile + G < tiles;
      const long long tn = more ? tile + G : tile;
      const int pn = int(tn / ctiles), cn = int(tn % ctiles) * 16;
      const double2* srcn = in + (size_t(pn) * b + cn) * Q;
      auto load_r = [&](int k, double2* r) {
        const int fz = par == 0 ? k : (k == 0 ? F : F - k);
        const double2* R =
            rhat + (k < iters && fz < F ? size_t(fz) * FF + pair : FF * F) * kRQ + p * kMaxQ + lk;
#pragma unroll
        for (int s = 0; s < kS; ++s) r[s] = R[4 * s];
      };
      auto products = [&](int k, const double2* r) {
        f64x4 c1 = {0.0, 0.0, 0.0, 0.0}, c2 = c1, c3 = c1;
#pragma unroll
        for (int s = 0; s < kS; ++s) {
          const double2 x = xf[k & 1][par][s][l];
          c1 = __builtin_amdgcn_mfma_f64_16x16x4f64(x.x, r[s].x, c1, 0, 0, 0);
          c2 = __builtin_amdgcn_mfma_f64_16x16x4f64(x.y, r[s].y, c2, 0, 0, 0);
          c3 = __builtin_amdgcn_mfma_f64_16x16x4f64(x.x + x.y, r[s].x + r[s].y, c3, 0, 0, 0);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v)
          yb[k & 1][par][j][v][l] = make_double2(c1[v] - c2[v], c3[v] - c1[v] - c2[v]);
      };
      // z-plane k of the next tile: 16 x kMaxQ elements, two per lane
      auto next_load = [&](int k, double2* g) {
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          const int e = tl + 256 * u, c = e / kMaxQ, q = e - c * kMaxQ;
          g[u] = more && q < Q && cn + c < b ? srcn[k * zstride + size_t(c) * Q + q]
                                            : make_double2(0.0, 0.0);
        }
      };
      auto next_store = [&](int k, const double2* g) {
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          const int e = tl + 256 * u, c = e / kMaxQ, q = e - c * kMaxQ;
          xn[(k * 16 + c) * QS + q] = g[u];
        }
      };
      double2 ra[kS], rb[kS], g[2];
      load_r(0, ra);
      int k = 0;
      for (; k + 2 <= iters; k += 2) {
        __syncthreads();  // xf[k & 1] complete, yb[k & 1] read
        next_load(k, g);
        load_r(k + 1, rb);
        products(k, ra);
        next_store(k, g);
        __syncthreads();
        next_load(k + 1, g);
        load_r(k + 2, ra);
        products(k + 1, rb);
        next_store(k + 1, g);
      }
      if (k < iters) {
        __syncthreads();
        next_load(k, g);
        products(k, ra);
        next_store(k, g);
      }
      __syncthreads();  // end of the tile
    }
    return;
  }
  // vector waves: elements (c = li, q = 4 s + lk), s = 2 vw + u, forward;
  // output elements e = 2 vw + u at (c = lk + 4 (e & 3), p = 16 (e >> 2) + li)
  const int vw = w - 4;
  for (long long tile = t0; tile < tiles; tile += G) {
    const int pair = int(tile / ctiles), c0 = int(tile % ctiles) * 16;
    double2 U[2][kT + 1], V[2][kT + 1];
    {
      double2 x[2][kW];
      if (tile == t0) {
        const bool rowok = c0 + li < b;
        const double2* src = in + (size_t(pair) * b + c0 + li) * Q;
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          const int q = 4 * (2 * vw + u) + lk;
          const bool ok = rowok && q < Q;
#pragma unroll
          for (int z = 0; z < kW; ++z)
            x[u][z] = ok ? src[z * zstride + q] : make_double2(0.0, 0.0);
        }
      } else {
        // staged by the matrix waves during the previous tile (zeros past
        // b and Q)
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
          for (int z = 0; z < kW; ++z) x[u][z] = xn[(z * 16 + li) * QS + 4 * (2 * vw + u) + lk];
      }
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        U[u][0] = x[u][kT];
        V[u][0] = make_double2(0.0, 0.0);
#pragma unroll
        for (int d = 1; d <= kT; ++d) {
          U[u][d] = make_double2(x[u][kT + d].x + x[u][kT - d].x, x[u][kT + d].y + x[u][kT - d].y);
          V[u][d] = make_double2(x[u][kT + d].x - x[u][kT - d].x, x[u][kT + d].y - x[u][kT - d].y);
        }
      }
    }
    auto fwd = [&](int k, int buf) {  // frequencies k and F - k of step k
      const double2* tf = Tf + size_t(k < F ? k : 0) * kW + kT;
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        double2 C = make_double2(0.0, 0.0), S = C;
#pragma unroll
        for (int d = 0; d <= kT; ++d) {
          const double2 m = tf[d];
          C.x = fma(m.x, U[u][d].x, C.x);
          C.y = fma(m.x, U[u][d].y, C.y);
          if (d > 0) {
            S.x = fma(m.y, V[u][d].x, S.x);
            S.y = fma(m.y, V[u][d].y, S.y);
          }
        }
        xf[buf][0][2 * vw + u][l] = make_double2(C.x - S.y, C.y + S.x);
        xf[buf][1][2 * vw + u][l] = make_double2(C.x + S.y, C.y - S.x);
      }
    };
    double2 P[2][kT + 1], M[2][kT + 1];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int d = 0; d <= kT; ++d) P[u][d] = M[u][d] = make_double2(0.0, 0.0);
    auto inv = [&](int k, int buf) {  // Y of step k (zero at k = -1)
      const double2* ti = Ti + size_t(kT) * F + (k > 0 ? k : 0);
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int e = 2 * vw + u;
        const double2 ya = yb[buf][0][e >> 2][e & 3][l], yc = yb[buf][1][e >> 2][e & 3][l];
        const double2 Sv = make_double2(ya.x + yc.x, ya.y + yc.y);
        const double2 Dv = make_double2(ya.x - yc.x, ya.y - yc.y);
#pragma unroll
        for (int d = 0; d <= kT; ++d) {
          const double2 m = ti[size_t(d) * F];
          P[u][d].x = fma(m.x, Sv.x, P[u][d].x);
          P[u][d].y = fma(m.x, Sv.y, P[u][d].y);
          if (d > 0) {
            M[u][d].x = fma(m.y, Dv.x, M[u][d].x);
            M[u][d].y = fma(m.y, Dv.y, M[u][d].y);
          }
        }
      }
    };
    // the Y of step -1 is zero (each lane reads back only what it wrote
    // here; the matrix waves write yb[1] first at step 1, after a barrier)
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int e = 2 * vw + u;
      yb[1][0][e >> 2][e & 3][l] = make_double2(0.0, 0.0);
      yb[1][1][e >> 2][e & 3][l] = make_double2(0.0, 0.0);
    }
    fwd(0, 0);
    for (int k = 0; k < iters; ++k) {
      __syncthreads();            // xf[k & 1] read next, yb[(k - 1) & 1] complete
      fwd(k + 1, (k + 1) & 1);  // unused after the last step
      inv(k - 1, (k - 1) & 1);
    }
    __syncthreads();  // end of the tile
    inv(iters - 1, (iters - 1) & 1);
    double2* dst = out + (size_t(pair) * b + c0) * Q;
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int e = 2 * vw + u;
      const int c = lk + 4 * (e & 3), pp = 16 * (e >> 2) + li;
      if (c0 + c < b && pp < Q) {
        double2* o = dst + size_t(c) * Q + pp;
        o[kT * zstride] = P[u][0];
#pragma unroll
        for (int d = 1; d <= kT; ++d) {
          o[(kT + d) * zstride] = make_double2(P[u][d].x - M[u][d].y, P[u][d].y + M[u][d].x);
          o[(kT - d) * zstride] = make_double2(P[u][d].x + M[u][d].y, P[u][d].y - M[u][d].x);
        }
      }
    }
  }
}

// One-axis transforms of the centred box through the frequency pairs (k,
// F - k) (as in k_tp_zfused), for the y passes: in[outer][W][inner] ->
// out[outer][F][inner] and back, one thread per (outer, inner) column.
template <int kW>
__global__ void __launch_bounds__(256) k_tp_fwd_pair(const double2* __restrict__ in,
                                                     const double2* __restrict__ Tf,
                                                     double2* __restrict__ out, long long outer,
                                                     long long inner) {
  constexpr int kT = kW / 2, kF = 2 * kW - 1;
  const long long idx = blockIdx.x * 256LL + threadIdx.x;
  if (idx >= outer * inner) return;
  const long long o = idx / inner, j = idx - o * inner;
  const double2* src = in + size_t(o) * kW * inner + j;
  double2 x[kW];
#pragma unroll
  for (int i = 0; i < kW; ++i) x[i] = src[size_t(i) * inner];
  double2 U[kT + 1], V[kT + 1];
  U[0] = x[kT];
  V[0] = make_double2(0.0, 0.0);
#pragma unroll
  for (int d = 1; d <= kT; ++d) {
    U[d] = make_double2(x[kT + d].x + x[kT - d].x, x[kT + d].y + x[kT - d].y);
    V[d] = make_double2(x[kT + d].x - x[kT - d].x, x[kT + d].y - x[kT - d].y);
  }
  double2* dst = out + size_t(o) * kF * inner + j;
#pragma unroll
  for (int k = 0; k <= 2 * kT; ++k) {
    const double2* tf = Tf + size_t(k) * kW + kT;
    double2 C = make_double2(0.0, 0.0), S = C;
#pragma unroll
    for (int d = 0; d <= kT; ++d) {
      const double2 m = tf[d];
      C.x = fma(m.x, U[d].x, C.x);
      C.y = fma(m.x, U[d].y, C.y);
      if (d > 0) {
        S.x = fma(m.y, V[d].x, S.x);
        S.y = fma(m.y, V[d].y, S.y);
      }
    }
    dst[size_t(k) * inner] = make_double2(C.x - S.y, C.y + S.x);
    if (k > 0) dst[size_t(kF - k) * inner] = make_double2(C.x + S.y, C.y - S.x);
  }
}

template <int kW>
__global__ void __launch_bounds__(256) k_tp_inv_pair(const double2* __restrict__ in,
                                                     const double2* __restrict__ Ti,
                                                     double2* __restrict__ out, long long outer,
                                                     long long inner) {
  constexpr int kT = kW / 2, kF = 2 * kW - 1;
  const long long idx = blockIdx.x * 256LL + threadIdx.x;
  if (idx >= outer * inner) return;
  const long long o = idx / inner, j = idx - o * inner;
  const double2* src = in + size_t(o) * kF * inner + j;
  double2 y[kF];
#pragma unroll
  for (int f = 0; f < kF; ++f) y[f] = src[size_t(f) * inner];
  double2 P[kT + 1], M[kT + 1];
#pragma unroll
  for (int d = 0; d <= kT; ++d) P[d] = M[d] = make_double2(0.0, 0.0);
#pragma unroll
  for (int k = 0; k <= 2 * kT; ++k) {
    const double2 ya = y[k], yc = k > 0 ? y[kF - k] : make_double2(0.0, 0.0);
    const double2 Sv = make_double2(ya.x + yc.x, ya.y + yc.y);
    const double2 Dv = make_double2(ya.x - yc.x, ya.y - yc.y);
#pragma unroll
    for (int d = 0; d <= kT; ++d) {
      const double2 m = Ti[size_t(kT + d) * kF + k];
      P[d].x = fma(m.x, Sv.x, P[d].x);
      P[d].y = fma(m.x, Sv.y, P[d].y);
      if (d > 0) {
        M[d].x = fma(m.y, Dv.x, M[d].x);
        M[d].y = fma(m.y, Dv.y, M[d].y);
      }
    }
  }
  double2* dst = out + size_t(o) * kW * inner + j;
  dst[size_t(kT) * inner] = P[0];
#pragma unroll
  for (int d = 1; d <= kT; ++d) {
    dst[size_t(kT + d) * inner] = make_double2(P[d].x - M[d].y, P[d].y + M[d].x);
    dst[size_t(kT - d) * inner] = make_double2(P[d].x + M[d].y, P[d].y - M[d].x);
  }
}

// A box row's support points are one run of consecutive support indices
// (lexicographic order, x fastest): cells x0 .. x0 + len - 1 <-> s0 ...
__device__ inline void row_run(const int* __restrict__ boxmap, int r, int W, int* x0, int* len,
                               int* s0) {
  int a = -1, n = 0, s = 0;
  for (int x = 0; x < W; ++x) {
    const int v = boxmap[r * W + x];
    if (v >= 0) {
      if (a < 0) {
        a = x;
        s = v;
      }
      ++n;
    }
  }
  *x0 = a < 0 ? 0 : a;
  *len = n;
  *s0 = s;
}

// Support block -> x spectrum of the box in one pass (the scatter onto the
// box and the x transform fused).  Workgroup = one box row r x 256 block
// elements e = c Q + q: the row's support run of each element (consecutive
// support indices, one contiguous run of the block's column) is loaded with
// consecutive lanes on consecutive points, staged in LDS, and each thread
// then transforms its element's row through the frequency pairs (k, F - k)
// of the centred box, as in k_tp_zfused, writing out[r][fx][e] along e.
// role 0: nothing to do (the gather copies X).
template <int kW>
__global__ void __launch_bounds__(256) k_tp_scatter_fx(const double2* __restrict__ X,
                                                       const int* __restrict__ boxmap,
                                                       const double2* __restrict__ Tf,
                                                       double2* __restrict__ out, int n, int L,
                                                       int Q, int b, int F,
                                                       const int* __restrict__ role) {
  constexpr int kT = kW / 2;
  __shared__ double2 vals[kW][256];
  if (role && *role == 0) return;
  const int bq = b * Q;
  const int r = blockIdx.y, e0 = blockIdx.x * 256;
  int x0, len, s0;
  row_run(boxmap, r, kW, &x0, &len, &s0);
  // vals[i][el] = X[c][q L + s0 + i] for the run, consecutive lanes along i
  for (int o = threadIdx.x; o < 256 * len; o += 256) {
    const int el = o / len, i = o - el * len, e = e0 + el;
    double2 v = make_double2(0.0, 0.0);
    if (e < bq) {
      const int c = e / Q, q = e - c * Q;
      v = X[size_t(c) * n + size_t(q) * L + s0 + i];
    }
    vals[i][el] = v;
  }
  __syncthreads();
  const int e = e0 + threadIdx.x;
  if (e >= bq) return;
  double2 x[kW];
#pragma unroll
  for (int i = 0; i < kW; ++i) {
    const int k = i - x0;
    x[i] = k >= 0 && k < len ? vals[k][threadIdx.x] : make_double2(0.0, 0.0);
  }
  double2 U[kT + 1], V[kT + 1];
  U[0] = x[kT];
  V[0] = make_double2(0.0, 0.0);
#pragma unroll
  for (int d = 1; d <= kT; ++d) {
    U[d] = make_double2(x[kT + d].x + x[kT - d].x, x[kT + d].y + x[kT - d].y);
    V[d] = make_double2(x[kT + d].x - x[kT - d].x, x[kT + d].y - x[kT - d].y);
  }
  double2* dst = out + size_t(r) * F * bq + e;
#pragma unroll
  for (int k = 0; k <= 2 * kT; ++k) {
    const double2* tf = Tf + size_t(k) * kW + kT;
    double2 C = make_double2(0.0, 0.0), S = C;
#pragma unroll
    for (int d = 0; d <= kT; ++d) {
      const double2 m = tf[d];
      C.x = fma(m.x, U[d].x, C.x);
      C.y = fma(m.x, U[d].y, C.y);
      if (d > 0) {
        S.x = fma(m.y, V[d].x, S.x);
        S.y = fma(m.y, V[d].y, S.y);
      }
    }
    dst[size_t(k) * bq] = make_double2(C.x - S.y, C.y + S.x);
    if (k > 0) dst[size_t(F - k) * bq] = make_double2(C.x + S.y, C.y - S.x);
  }
}

// x spectrum of the box -> support block in one pass (the inverse x
// transform and the gather fused).  Workgroup = one box row r x 256 block
// elements: each thread reads its element's F frequencies (along e, as
// written), forms the row's box values through the frequency pairs and puts
// the row's support run in LDS; then the run of every element is written,
// consecutive lanes on consecutive support points: out[c][q L + s] = S, or
// a S + bc X + g prev with (a, bc, g) = coef[0..2] (coef[3..5] for role 2);
// role 0 copies X.  Every support point lies in exactly one box row.
template <int kW>
__global__ void __launch_bounds__(256) k_tp_ix_gather(const double2* __restrict__ in,
                                                      const int* __restrict__ boxmap,
                                                      const double2* __restrict__ Ti,
                                                      const double2* __restrict__ X,
                                                      double2* out, const double2* prev, int n,
                                                      int L, int Q, int b,
                                                      const double* __restrict__ coef,
                                                      const int* __restrict__ role) {
  constexpr int kT = kW / 2, kF = 2 * kW - 1;
  __shared__ double2 vals[kW][256];
  const int bq = b * Q;
  const int r = blockIdx.y, e0 = blockIdx.x * 256;
  int x0, len, s0;
  row_run(boxmap, r, kW, &x0, &len, &s0);
  int rl = 1;
  if (role) {
    rl = *role;
    if (rl == 2) coef += 3;
  }
  const int e = e0 + threadIdx.x;
  if (rl != 0 && e < bq) {
    double2 y[kF];
    const double2* src = in + size_t(r) * kF * bq + e;
#pragma unroll
    for (int f = 0; f < kF; ++f) y[f] = src[size_t(f) * bq];
    double2 P[kT + 1], M[kT + 1];
#pragma unroll
    for (int d = 0; d <= kT; ++d) P[d] = M[d] = make_double2(0.0, 0.0);
#pragma unroll
    for (int k = 0; k <= 2 * kT; ++k) {
      const double2 ya = y[k], yc = k > 0 ? y[kF - k] : make_double2(0.0, 0.0);
      const double2 Sv = make_double2(ya.x + yc.x, ya.y + yc.y);
      const double2 Dv = make_double2(ya.x - yc.x, ya.y - yc.y);
#pragma unroll
      for (int d = 0; d <= kT; ++d) {
        const double2 m = Ti[size_t(kT + d) * kF + k];
        P[d].x = fma(m.x, Sv.x, P[d].x);
        P[d].y = fma(m.x, Sv.y, P[d].y);
        if (d > 0) {
          M[d].x = fma(m.y, Dv.x, M[d].x);
          M[d].y = fma(m.y, Dv.y, M[d].y);
        }
      }
    }
#pragma unroll
    for (int i = 0; i < kW; ++i) {
      const int k = i - x0;
      if (k < 0 || k >= len) continue;
      const int d = i - kT, ad = d < 0 ? -d : d;
      const double sg = d < 0 ? -1.0 : 1.0;
      vals[k][threadIdx.x] = d == 0 ? P[0]
                                    : make_double2(P[ad].x - sg * M[ad].y, P[ad].y + sg * M[ad].x);
    }
  }
  __syncthreads();
  for (int o = threadIdx.x; o < 256 * len; o += 256) {
    const int el = o / len, i = o - el * len, ee = e0 + el;
    if (ee >= bq) continue;
    const int c = ee / Q, q = ee - c * Q;
    const size_t idx = size_t(c) * n + size_t(q) * L + s0 + i;
    if (rl == 0) {
      out[idx] = X[idx];
      continue;
    }
    const double2 v = vals[i][el];
    double2 res = v;
    if (coef) {
      const double2 xv = X[idx];
      res = make_double2(coef[0] * v.x + coef[1] * xv.x, coef[0] * v.y + coef[1] * xv.y);
      if (prev) {
        const double2 pv = prev[idx];
        res.x += coef[2] * pv.x;
        res.y += coef[2] * pv.y;
      }
    }
    out[idx] = res;
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

size_t toeplitz_rhat_elems(const Plan& p) {
  return (size_t(p.K[0]) * p.K[1] * p.K[2] + 1) * kRQ;
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
  PISCO_KERNEL(h, k_tp_rhat, dim3(ceil_div((nf + 1) * kRQ, 256)), dim3(256), 0, lf, op.rhat,
               op.Q, nf);
  return PISCO_OK;
}

pisco_status_t toeplitz_product(Handle* h, const ToeplitzOp& op, const double2* X,
                                double2* out, int n, int b, const double* coef,
                                const double2* prev, const int* role) {
  const int Q = op.Q, W = op.W, Wz = op.Wz, F = op.F, Fz = op.Fz;
  const int bq = b * Q;
  const int cells = Wz * W * W, rows = Wz * W;
  // the box's x passes fused with the scatter and the gather for the box
  // widths with a compiled kernel
  const bool fused_x = (W & 1) && W >= 3 && W <= 13 && F == 2 * W - 1;
  pisco_status_t st;
  // box -> frequency: x (into buf1), y (, z)
  if (fused_x) {
    switch (W) {
#define TP_SX(w)                                                                                \
  case w:                                                                                       \
    PISCO_KERNEL(h, k_tp_scatter_fx<w>, dim3(ceil_div(bq, 256), rows), dim3(256), 0, X,         \
                 op.boxmap, op.Tf, op.buf1, n, op.L, Q, b, F, role);                            \
    break;
      TP_SX(3) TP_SX(5) TP_SX(7) TP_SX(9) TP_SX(11) TP_SX(13)
#undef TP_SX
    }
  } else {
    PISCO_KERNEL(h, k_tp_scatter, dim3(ceil_div(1LL * cells * bq, 256)), dim3(256), 0, X,
                 op.boxmap, op.buf0, n, op.L, Q, b, cells, role);
    const int fx[4] = {rows, W, bq, 1};
    if ((st = axis_transform64(h, op.buf0, op.buf1, fx, 1, F, op.Tf))) return st;
  }
  const long long yin = 1LL * F * bq;  // inner extent of the y passes
  if (fused_x) {
    switch (W) {
#define TP_FY(w)                                                                                \
  case w:                                                                                       \
    PISCO_KERNEL(h, k_tp_fwd_pair<w>, dim3(ceil_div(Wz * yin, 256)), dim3(256), 0, op.buf1,     \
                 op.Tf, op.buf0, (long long)Wz, yin);                                           \
    break;
      TP_FY(3) TP_FY(5) TP_FY(7) TP_FY(9) TP_FY(11) TP_FY(13)
#undef TP_FY
    }
  } else {
    const int fy[4] = {Wz, W, F * bq, 1};
    if ((st = axis_transform64(h, op.buf1, op.buf0, fy, 1, F, op.Tf))) return st;
  }
  // per-frequency products; the y spectrum of the box ends in `ys`
  double2* ys = op.buf0;
  if (op.D == 3 && (W & 1) && W >= 3 && W <= 11 && Fz == F && Wz == W) {
    // z pass, per-frequency products and inverse z pass fused: buf0 -> buf1
    // a persistent grid: one workgroup per CU, each walking a range of tiles
    const int ctiles = ceil_div(b, 16);
    const int tiles = F * F * ctiles;
    const dim3 grid(unsigned(tiles < h->num_cu ? tiles : h->num_cu));
    const dim3 blk(512);
    switch (W) {
#define TP_ZF(w)                                                                                 \
  case w:                                                                                        \
    PISCO_KERNEL(h, k_tp_zfused<w>, grid, blk, 0, op.buf0, op.rhat, op.Tf, op.Ti, op.buf1, Q, b, \
                 F, ctiles, tiles, role);                                                        \
    break;
      TP_ZF(3) TP_ZF(5) TP_ZF(7) TP_ZF(9) TP_ZF(11)
#undef TP_ZF
    }
    switch (W) {
#define TP_IY(w)                                                                                \
  case w:                                                                                       \
    PISCO_KERNEL(h, k_tp_inv_pair<w>, dim3(ceil_div(Wz * yin, 256)), dim3(256), 0, op.buf1,     \
                 op.Ti, op.buf0, (long long)Wz, yin);                                           \
    break;
      TP_IY(3) TP_IY(5) TP_IY(7) TP_IY(9) TP_IY(11)
#undef TP_IY
    }
    ys = op.buf0;
  } else {
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
    // frequency -> box: (z,) y
    double2* cur = other;
    double2* nxt = spec;
    if (op.D == 3) {
      const int iz[4] = {1, Fz, F * F * bq, 1};
      if ((st = axis_transform64(h, cur, nxt, iz, 1, Wz, op.Ti))) return st;
      double2* tmp = cur;
      cur = nxt;
      nxt = tmp;
    }
    if (fused_x) {
      switch (W) {
#define TP_IY(w)                                                                                \
  case w:                                                                                       \
    PISCO_KERNEL(h, k_tp_inv_pair<w>, dim3(ceil_div(Wz * yin, 256)), dim3(256), 0, cur, op.Ti,  \
                 nxt, (long long)Wz, yin);                                                      \
    break;
        TP_IY(3) TP_IY(5) TP_IY(7) TP_IY(9) TP_IY(11) TP_IY(13)
#undef TP_IY
      }
    } else {
      const int iy[4] = {Wz, F, F * bq, 1};
      if ((st = axis_transform64(h, cur, nxt, iy, 1, W, op.Ti))) return st;
    }
    ys = nxt;
  }
  // x back and the support points, with the epilogue
  if (fused_x) {
    switch (W) {
#define TP_XG(w)                                                                                 \
  case w:                                                                                        \
    PISCO_KERNEL(h, k_tp_ix_gather<w>, dim3(ceil_div(bq, 256), rows), dim3(256), 0, ys,          \
                 op.boxmap, op.Ti, X, out, prev, n, op.L, Q, b, coef, role);                     \
    break;
      TP_XG(3) TP_XG(5) TP_XG(7) TP_XG(9) TP_XG(11) TP_XG(13)
#undef TP_XG
    }
    return PISCO_OK;
  }
  double2* box = ys == op.buf0 ? op.buf1 : op.buf0;
  const int ix[4] = {rows, F, bq, 1};
  if ((st = axis_transform64(h, ys, box, ix, 1, W, op.Ti))) return st;
  PISCO_KERNEL(h, k_tp_gather, dim3(ceil_div(1LL * b * n, 256)), dim3(256), 0, box, op.sup, X,
               out, prev, n, op.L, Q, b, W, op.D == 3 ? op.W / 2 : 0, op.W / 2, coef, role);
  return PISCO_OK;
}

}  // namespace pisco
