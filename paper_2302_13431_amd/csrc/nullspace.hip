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
//        block staying well conditioned, and such a chain applies a
//        Chebyshev polynomial of A that damps everything below the block;
// and, when an error model built from the Cholesky diagonal (about the
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

// Z = A X, A float2 row-major n x n (widened exactly to FP64), X and Z
// column-major n x b (double2).  One wave per 32 x 32 output tile and K
// slice, on FP64 matrix cores: each complex
// 16 x 16 x 4 block step is three real v_mfma_f64_16x16x4f64 products, the
// three-multiplication form of a complex product: T1 += Ar Xr, T2 += Ai Xi,
// T3 += (Ar + Ai)(Xr + Xi), and at the end Re = T1 - T2, Im = T3 - T1 - T2
// (a quarter fewer matrix-core products than Re += Ar Xr - Ai Xi, Im += Ar
// Xi + Ai Xr; the rounding error stays of order eps sum |A||X|).  Operand lanes: lane l
// supplies row (or column) l % 16 at k = k0 + 4 s + l / 16 for step s, so a
// lane's four k of one chunk are 4 apart and every load instruction reads
// 4 consecutive elements per row; accumulator element v of lane l is row
// l / 16 + 4 v, column l % 16.  Operands for the next chunk of 16 k are
// loaded before the products of the current one, into the other of two
// buffers.  Every wave reads only its own rows of A, so the three column
// tiles of a row share A through the caches.
typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int kAxQ = 4;           // k steps of 4 per operand chunk
constexpr int kAxK = 4 * kAxQ;    // k per chunk
struct AxChunk {
  float2 a[2][kAxQ];    // rows r0 + li (+16), k = k0 + 4 q + lk
  double2 x[2][kAxQ];   // columns c0 + li (+16), same k
};

// A whole chunk inside the slice: one base address per row and column and
// constant offsets (rows past n read row 0 of the tile and are zeroed).
__device__ inline void ax_load_full(AxChunk& ch, const float2* Ar0, const float2* Ar1, bool v0,
                                    bool v1, const double2* X0, const double2* X1, int k0,
                                    int lk) {
  const float2* a0 = Ar0 + k0 + lk;
  const float2* a1 = Ar1 + k0 + lk;
  const double2* x0 = X0 + k0 + lk;
  const double2* x1 = X1 + k0 + lk;
#pragma unroll
  for (int q = 0; q < kAxQ; ++q) {
    const float2 u0 = a0[4 * q], u1 = a1[4 * q];
    ch.a[0][q] = make_float2(v0 ? u0.x : 0.f, v0 ? u0.y : 0.f);
    ch.a[1][q] = make_float2(v1 ? u1.x : 0.f, v1 ? u1.y : 0.f);
    ch.x[0][q] = x0[4 * q];
    ch.x[1][q] = x1[4 * q];
  }
}

// The last, partial chunk of a slice, branch-free: every lane loads from a
// valid address (k clamped to the slice) and the value is zeroed after.
__device__ inline void ax_load(AxChunk& ch, const float2* Ar0, const float2* Ar1, bool v0,
                               bool v1, const double2* X0, const double2* X1, int k0, int lk,
                               int kend) {
#pragma unroll
  for (int q = 0; q < kAxQ; ++q) {
    const int k = k0 + 4 * q + lk;
    const bool ok = k < kend;
    const int kk = ok ? k : kend - 1;
    const float2 a0 = Ar0[kk], a1 = Ar1[kk];
    const double2 x0 = X0[kk], x1 = X1[kk];
    ch.a[0][q] = make_float2(ok && v0 ? a0.x : 0.f, ok && v0 ? a0.y : 0.f);
    ch.a[1][q] = make_float2(ok && v1 ? a1.x : 0.f, ok && v1 ? a1.y : 0.f);
    ch.x[0][q] = make_double2(ok ? x0.x : 0.0, ok ? x0.y : 0.0);
    ch.x[1][q] = make_double2(ok ? x1.x : 0.0, ok ? x1.y : 0.0);
  }
}

// The kKS K slices of one tile are the kKS waves of one workgroup: each
// leaves its 32 x 32 partial in LDS (column stride 33: no bank conflicts),
// and the workgroup adds them in slice order (deterministic) and writes
// out = a S + bc Y + g P with (a, bc, g) = coef[0..2] (Chebyshev steps; Y =
// the block multiplied, P = prev, may be null) or out = S when coef is
// null.  out may be prev (each element is read before it is written by the
// same thread) but not X.
template <int kKS>
__global__ void __launch_bounds__(64 * kKS) __attribute__((amdgpu_waves_per_eu(2))) k_gemm_ax(const float2* __restrict__ A,
                                                      const double2* __restrict__ X,
                                                      double2* out, int n, int b, int kchunk,
                                                      const double* __restrict__ coef,
                                                      const double2* prev,
                                                      const int* __restrict__ role) {
  __shared__ double2 red[kKS > 1 ? kKS * 32 * 33 : 1];
  const int l = threadIdx.x & 63;
  const int z = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int li = l & 15, lk = l >> 4;
  // Workgroups go to the eight XCDs in turn (linear id mod 8).  Tiles are
  // dealt so that each XCD runs one contiguous range, row tile by row tile
  // with its column tiles adjacent: the column tiles of a row tile then run
  // together on one XCD and share the rows of A they read in its L2.
  int r0, c0;
  {
    const int ntx = gridDim.x, nty = gridDim.y, total = ntx * nty;
    const int id = blockIdx.x + ntx * blockIdx.y;
    const int xcd = id % 8, slot = id / 8;
    const int base = total / 8, extra = total % 8;
    const int tile = xcd * base + (xcd < extra ? xcd : extra) + slot;
    r0 = (tile / nty) * 32;
    c0 = (tile % nty) * 32;
  }
  if (role) {
    // device-resident schedule: the slot's role is decided on the device
    // (0: skipped, the block is copied so that the buffers keep their
    // roles; 1: first step of a chain, coef[0..2]; 2: later step, coef[3..5])
    const int r = __builtin_amdgcn_readfirstlane(*role);
    if (r == 0) {
      for (int e = threadIdx.x; e < 32 * 32; e += 64 * kKS) {
        const int row = e & 31, col = e >> 5;
        if (r0 + row < n) out[size_t(c0 + col) * n + r0 + row] = X[size_t(c0 + col) * n + r0 + row];
      }
      return;
    }
    if (r == 2) coef += 3;
  }
  const int kbeg = z * kchunk;
  const int kend = min(n, kbeg + kchunk);
  const bool v0 = r0 + li < n, v1 = r0 + 16 + li < n;
  const float2* Ar0 = A + size_t(v0 ? r0 + li : 0) * n;
  const float2* Ar1 = A + size_t(v1 ? r0 + 16 + li : 0) * n;
  const double2* X0 = X + size_t(c0 + li) * n;
  const double2* X1 = X + size_t(c0 + 16 + li) * n;
  f64x4 t1[2][2], t2[2][2], t3[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      t1[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};
      t2[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};
      t3[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};
    }
  // the twelve accumulators are updated in turn, so that two products
  // into one accumulator are never back to back
  auto mma = [&](const AxChunk& cur) {
#pragma unroll
    for (int s = 0; s < kAxQ; ++s) {
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const double ar = cur.a[i][s].x, ai = cur.a[i][s].y, as = ar + ai;
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          const double xr = cur.x[j][s].x, xi = cur.x[j][s].y;
          t1[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, xr, t1[i][j], 0, 0, 0);
          t2[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, xi, t2[i][j], 0, 0, 0);
          t3[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(as, xr + xi, t3[i][j], 0, 0, 0);
        }
      }
    }
  };
  // two operand buffers in turn (a copy from one to the other would make
  // the copy wait for the loads just issued): the next chunk's loads are in
  // flight while the current chunk's products run
  // complete chunks in the loop, a partial last one after it
  auto load = [&](AxChunk& ch, int k0) { ax_load_full(ch, Ar0, Ar1, v0, v1, X0, X1, k0, lk); };
  const int kfull = kend > kbeg ? kbeg + (kend - kbeg) / kAxK * kAxK : kbeg;
  AxChunk q0, q1;
  if (kfull > kbeg) {
    // loads unconditional (past the end they repeat the last chunk,
    // unused): no branch, so each product waits only for its own buffer
    const int klast = kfull - kAxK;
    load(q0, kbeg);
    for (int k0 = kbeg; k0 < kfull; k0 += 2 * kAxK) {
      load(q1, min(k0 + kAxK, klast));
      mma(q0);
      if (k0 + kAxK >= kfull) break;
      load(q0, min(k0 + 2 * kAxK, klast));
      mma(q1);
    }
  }
  if (kfull < kend) {
    ax_load(q0, Ar0, Ar1, v0, v1, X0, X1, kfull, lk, kend);
    mma(q0);
  }
  f64x4 cr[2][2], ci[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        cr[i][j][v] = t1[i][j][v] - t2[i][j][v];
        ci[i][j][v] = t3[i][j][v] - t1[i][j][v] - t2[i][j][v];
      }
  // partial tile -> LDS slot z (row 16 i + lk + 4 v, column 16 j + li)
  double2* slot = red + (kKS > 1 ? z * 32 * 33 : 0);
  if (kKS > 1) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          slot[(16 * j + li) * 33 + 16 * i + lk + 4 * v] = make_double2(cr[i][j][v], ci[i][j][v]);
    __syncthreads();
  }
  double a = 1.0, bc = 0.0, g = 0.0;
  if (coef) {
    a = coef[0];
    bc = coef[1];
    g = coef[2];
  }
  auto emit = [&](int row, int col, double2 sum) {
    const size_t o = size_t(c0 + col) * n + r0 + row;
    double2 r = sum;
    if (coef) {
      const double2 y = X[o];
      r = make_double2(a * sum.x + bc * y.x, a * sum.y + bc * y.y);
      if (prev) {
        const double2 q = prev[o];
        r.x += g * q.x;
        r.y += g * q.y;
      }
    }
    out[o] = r;
  };
  if (kKS > 1) {
    for (int e = threadIdx.x; e < 32 * 32; e += 64 * kKS) {
      const int row = e & 31, col = e >> 5;
      if (r0 + row >= n) continue;
      double2 sum = red[col * 33 + row];
#pragma unroll
      for (int q = 1; q < kKS; ++q) sum = zadd(sum, red[q * 32 * 33 + col * 33 + row]);
      emit(row, col, sum);
    }
  } else {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = 16 * i + lk + 4 * v, col = 16 * j + li;
          if (r0 + row < n) emit(row, col, make_double2(cr[i][j][v], ci[i][j][v]));
        }
  }
}

// out = sum over `parts` slabs of size `len` (fixed order: deterministic).
// The slabs are read 24 at a time, all of those loads in flight together;
// workgroups of one wave spread the few thousand elements over many CUs.
__global__ void __launch_bounds__(64) k_sum_parts(const double2* __restrict__ parts,
                                                  double2* __restrict__ out, long long len,
                                                  int nparts, const int* __restrict__ skip) {
  if (skip && *skip) return;
  constexpr int kU = 24;
  const long long i = blockIdx.x * 64LL + threadIdx.x;
  if (i >= len) return;
  double2 s = make_double2(0.0, 0.0);
  for (int k0 = 0; k0 < nparts; k0 += kU) {
    double2 v[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u)
      v[u] = k0 + u < nparts ? parts[size_t(k0 + u) * len + i] : make_double2(0.0, 0.0);
#pragma unroll
    for (int u = 0; u < kU; ++u)
      if (k0 + u < nparts) s = zadd(s, v[u]);
  }
  out[i] = s;
}

// part[chunk] = P[rows of chunk, :]^H Q[rows of chunk, :]; P, Q column-major
// n x b (b a multiple of 16); part is column-major b x b.  Rows are split
// in chunks of kTnRows.  One wave per 16 x 16 block of the result and row
// chunk, on FP64 matrix cores (operand and accumulator lanes as in
// k_gemm_ax): Re += Pr Qr + Pi Qi, Im += Pr Qi - Pi Qr.  With upper, blocks
// below the diagonal are skipped (their entries of part are left as they
// are).  The rows of the next 16 are loaded before the products of the
// current ones; even and odd steps go to separate accumulators.
__global__ void __launch_bounds__(64) k_gemm_tn(const double2* __restrict__ P,
                                                const double2* __restrict__ Qm,
                                                double2* __restrict__ part, int n, int b,
                                                int upper, const int* __restrict__ skip) {
  if (upper && blockIdx.x > blockIdx.y) return;
  if (skip && *skip) return;
  const int l = threadIdx.x, li = l & 15, lk = l >> 4;
  const int i0 = blockIdx.x * 16, j0 = blockIdx.y * 16;
  const int rbeg = blockIdx.z * kTnRows, rend = min(n, rbeg + kTnRows);
  const double2* Pc = P + size_t(i0 + li) * n;
  const double2* Qc = Qm + size_t(j0 + li) * n;
  // three real products per complex step: with a = Pr, b = -Pi, c = Qr,
  // d = Qi, conj(P) Q = (ac - bd) + i((a + b)(c + d) - ac - bd)
  f64x4 t1[2], t2[2], t3[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) t1[h] = t2[h] = t3[h] = f64x4{0.0, 0.0, 0.0, 0.0};
  // two operand buffers in turn (a copy from one to the other would make
  // the copy wait for the loads just issued); complete steps of 16 rows in
  // the loop with plain loads, a partial last one after it (rows clamped
  // and zeroed: predicated loads, or a zeroing select at load time, would
  // make the products wait for every load in flight)
  double2 pa[4], qa[4], pb[4], qb[4];
  auto load = [&](int r0, double2 (&p)[4], double2 (&q)[4]) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      p[u] = Pc[r0 + 4 * u + lk];
      q[u] = Qc[r0 + 4 * u + lk];
    }
  };
  auto mma = [&](const double2 (&pv)[4], const double2 (&qv)[4]) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const double2 x = pv[u], y = qv[u];
      t1[u & 1] = __builtin_amdgcn_mfma_f64_16x16x4f64(x.x, y.x, t1[u & 1], 0, 0, 0);
      t2[u & 1] = __builtin_amdgcn_mfma_f64_16x16x4f64(-x.y, y.y, t2[u & 1], 0, 0, 0);
      t3[u & 1] = __builtin_amdgcn_mfma_f64_16x16x4f64(x.x - x.y, y.x + y.y, t3[u & 1], 0, 0, 0);
    }
  };
  const int rfull = rend > rbeg ? rbeg + (rend - rbeg) / 16 * 16 : rbeg;
  if (rfull > rbeg) {
    // loads unconditional (past the end they repeat the last step, unused):
    // no branch, so each product waits only for its own buffer
    const int rlast = rfull - 16;
    load(rbeg, pa, qa);
    for (int r0 = rbeg; r0 < rfull; r0 += 32) {
      load(min(r0 + 16, rlast), pb, qb);
      mma(pa, qa);
      if (r0 + 16 >= rfull) break;
      load(min(r0 + 32, rlast), pa, qa);
      mma(pb, qb);
    }
  }
  if (rfull < rend) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int r = rfull + 4 * u + lk;
      const bool ok = r < rend;
      const int rr = ok ? r : rend - 1;
      const double2 x = Pc[rr], y = Qc[rr];
      pa[u] = make_double2(ok ? x.x : 0.0, ok ? x.y : 0.0);
      qa[u] = make_double2(ok ? y.x : 0.0, ok ? y.y : 0.0);
    }
    mma(pa, qa);
  }
  double2* out = part + size_t(blockIdx.z) * b * b;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int row = i0 + lk + 4 * e, col = j0 + li;
    const double a = t1[0][e] + t1[1][e], c = t2[0][e] + t2[1][e], d = t3[0][e] + t3[1][e];
    out[size_t(col) * b + row] = make_double2(a - c, d - a - c);
  }
}

// Y = P M; P column-major m x k, M column-major k x b, Y column-major m x b
// (b a multiple of 16).  One wave per 16 x 16 tile of Y on FP64 matrix cores
// (Re += Pr Mr - Pi Mi, Im += Pr Mi + Pi Mr), so that a block of b = 96
// columns gives 6 m / 16 waves.  With tri, M is upper triangular and the
// sum over k stops at the tile's last column.  The operands of the next 16
// k are loaded before the products of the current ones; even and odd steps
// of 4 k go to separate accumulators.
__global__ void __launch_bounds__(64) k_gemm_nn(const double2* __restrict__ Pm,
                                                const double2* __restrict__ M,
                                                double2* __restrict__ Y, int m, int k,
                                                int b, int tri, const int* __restrict__ copy) {
  const int l = threadIdx.x, li = l & 15, lk = l >> 4;
  const int r0 = blockIdx.x * 16, c0 = blockIdx.y * 16;
  if (copy && *copy) {
    // skipped orthonormalisation (k == b): Y = P, so the buffers keep their roles
    for (int e = l; e < 256; e += 64) {
      const int row = r0 + (e & 15), col = c0 + (e >> 4);
      if (row < m) Y[size_t(col) * m + row] = Pm[size_t(col) * m + row];
    }
    return;
  }
  const bool v = r0 + li < m;
  const int kend = tri ? min(k, c0 + 16) : k;
  const double2* Mc = M + size_t(c0 + li) * k;
  const double2* Pr = Pm + (v ? r0 + li : 0);
  // three real products per complex step: T1 = Pr Mr, T2 = Pi Mi,
  // T3 = (Pr + Pi)(Mr + Mi); Re = T1 - T2, Im = T3 - T1 - T2
  f64x4 t1[2], t2[2], t3[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) t1[h] = t2[h] = t3[h] = f64x4{0.0, 0.0, 0.0, 0.0};
  // two operand buffers in turn (a copy from one to the other would make
  // the copy wait for the loads just issued); complete steps of 16 k in the
  // loop with unconditional loads (past the end they repeat the last step,
  // unused: no branch, so each product waits only for its own buffer), a
  // partial last step after it (k clamped and zeroed); rows past m read row
  // 0 of the tile and are zeroed where they are stored
  double2 pa[4], ma[4], pb[4], mb[4];
  auto load = [&](int k0, double2 (&p)[4], double2 (&q)[4]) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int kk = k0 + 4 * u + lk;
      p[u] = Pr[size_t(kk) * m];
      q[u] = Mc[kk];
    }
  };
  auto mma = [&](const double2 (&pv)[4], const double2 (&mv)[4]) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const double2 x = pv[u], y = mv[u];
      t1[u & 1] = __builtin_amdgcn_mfma_f64_16x16x4f64(x.x, y.x, t1[u & 1], 0, 0, 0);
      t2[u & 1] = __builtin_amdgcn_mfma_f64_16x16x4f64(x.y, y.y, t2[u & 1], 0, 0, 0);
      t3[u & 1] = __builtin_amdgcn_mfma_f64_16x16x4f64(x.x + x.y, y.x + y.y, t3[u & 1], 0, 0, 0);
    }
  };
  const int kfull = kend / 16 * 16;
  if (kfull > 0) {
    const int klast = kfull - 16;
    load(0, pa, ma);
    for (int k0 = 0; k0 < kfull; k0 += 32) {
      load(min(k0 + 16, klast), pb, mb);
      mma(pa, ma);
      if (k0 + 16 >= kfull) break;
      load(min(k0 + 32, klast), pa, ma);
      mma(pb, mb);
    }
  }
  if (kfull < kend) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int kk = kfull + 4 * u + lk;
      const bool ok = kk < kend;
      const int kc = ok ? kk : kend - 1;
      const double2 x = Pr[size_t(kc) * m], y = Mc[kc];
      pa[u] = make_double2(ok ? x.x : 0.0, ok ? x.y : 0.0);
      ma[u] = make_double2(ok ? y.x : 0.0, ok ? y.y : 0.0);
    }
    mma(pa, ma);
  }
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int row = r0 + lk + 4 * e, col = c0 + li;
    const double a = t1[0][e] + t1[1][e], c = t2[0][e] + t2[1][e], d = t3[0][e] + t3[1][e];
    if (row < m) Y[size_t(col) * m + row] = make_double2(a - c, d - a - c);
  }
}

__device__ inline double readlane_f64(double v, int lane) {
  const long long x = __double_as_longlong(v);
  const unsigned lo = __builtin_amdgcn_readlane(int(x), lane);
  const unsigned hi = __builtin_amdgcn_readlane(int(x >> 32), lane);
  return __longlong_as_double((static_cast<long long>(hi) << 32) | lo);
}

// ------------------------------------------------------------------ Cholesky QR

constexpr int kCholLdsMax = 96;  // largest b factored with the matrix in LDS
constexpr int kCholThreads = 1024;

// Cholesky factor of D S D + shift I, D = diag(S)^{-1/2}: R (upper, column-
// major b x b, entries below the diagonal zero) and D itself (dsc), so that
// Y D R^{-1} has orthonormal columns when S = Y^H Y (up to the shift).  One
// workgroup; the working matrix T (row-major, ld = b + 1 so that column
// walks spread over the LDS banks) is in LDS when kLds (b <= 96) and in
// `gwork` otherwise.  A pivot that is not positive is replaced by a tiny
// one and reported through *flag.
//
// Blocked in panels of kNB = 8 rows (b must be a multiple).  Per panel J
// the block row T_J,J: is eliminated right-looking, one column per lane:
// lanes 0..7 of a wave hold the diagonal block's columns, lanes 8..63 a
// group of 56 later columns, each lane its column's 8 panel entries in
// registers.  Step k takes the pivot and row k of the diagonal block from
// lanes 0..7 by readlane, so the 8 steps run without barriers or LDS
// round trips; every wave that owns a column group repeats the diagonal
// lanes.  The finished block row R_J,: goes straight to R, and its part
// right of the diagonal block to LDS for the trailing update.
// After a barrier the trailing update T_ij -= R_Ji^H R_Jj runs in 2 x 2
// patches of the upper triangle, one per thread, operands in registers.
//
// Blocked use (kLds false, large b): a call eliminates only the panels of
// rows [kbeg, kend) and applies their trailing updates to those rows alone
// (every column right of the diagonal); the update of the rows below, with
// the finished rows R_[kbeg,kend),: as one rank-(kend - kbeg) block, is
// k_chol_update's, across many workgroups.  T, the scales and R's lower
// part are staged beforehand by k_chol_stage; every call reads the scales
// back from dsc_out.
template <bool kLds>
__global__ void __launch_bounds__(kCholThreads) k_chol(const double2* __restrict__ S, int b,
                                               double shift, double2* __restrict__ R,
                                               double* __restrict__ dsc_out,
                                               double2* __restrict__ gwork,
                                               int* __restrict__ flag,
                                               double* __restrict__ rdiag,
                                               const int* __restrict__ skip, int kbeg,
                                               int kend) {
  if (skip && *skip) return;
  constexpr int kNB = 8;                        // panel height (b is a multiple)
  constexpr int kNT = kCholThreads;
  constexpr int kCols = 64 - kNB;               // later columns per wave and group
  __shared__ double2 lds_mat[kLds ? kCholLdsMax * (kCholLdsMax + 1) : 1];
  __shared__ double dsc[kLds ? kCholLdsMax : 1024];
  double2* T = kLds ? lds_mat : gwork;
  const int ld = b + 1;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  auto at = [&](int i, int j) -> double2& { return T[i * ld + j]; };
  // S and R are column-major.  The upper triangle of T is staged here and
  // the part of R below the diagonal zeroed, in a loop of its own (merged
  // into one branch, the two kinds of store become flat stores that wait
  // on memory); the rest of R is written per panel
  auto stage = [&](int i, int j, double2 v) {
    if (j < i) return;
    v = zscale(v, dsc[i] * dsc[j]);
    if (i == j) v = make_double2(v.x + shift, 0.0);
    at(i, j) = v;
  };
  auto zero_lower = [&](int i, int j) {
    if (j < i) R[size_t(j) * b + i] = make_double2(0.0, 0.0);
  };
  if constexpr (kLds) {
    // every load in flight at once, before the scales are known
    constexpr int kPer = (kCholLdsMax * kCholLdsMax + kNT - 1) / kNT;
    double2 v[kPer];
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int e = t + kNT * q;
      v[q] = e < b * b ? S[e] : make_double2(0.0, 0.0);
    }
    if (t < b) {
      const double d = S[size_t(t) * b + t].x;
      dsc[t] = d > 0.0 ? 1.0 / sqrt(d) : 0.0;
      dsc_out[t] = dsc[t];
    }
    __syncthreads();
    // element e = t + kNT q is (i, j) = (e mod b, e div b), stepped
    // without a division per element
    const int di = kNT % b, dj = kNT / b;
    int i = t % b, j = t / b;
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      if (t + kNT * q < b * b) stage(i, j, v[q]);
      i += di;
      j += dj;
      if (i >= b) {
        i -= b;
        ++j;
      }
    }
    i = t % b;
    j = t / b;
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      if (t + kNT * q < b * b) zero_lower(i, j);
      i += di;
      j += dj;
      if (i >= b) {
        i -= b;
        ++j;
      }
    }
  } else {
    // blocked use: T, the scales and R's lower part were staged by
    // k_chol_stage across many workgroups
    for (int k = t; k < b; k += kNT) dsc[k] = dsc_out[k];
  }
  __syncthreads();
  for (int k0 = kbeg; k0 < kend; k0 += kNB) {
    const int k1 = k0 + kNB, nc = b - k1;
    const int groups = nc > 0 ? (nc + kCols - 1) / kCols : 1;
    for (int g = wave; g < groups; g += kNT / 64) {
      const int c = lane < kNB ? k0 + lane : k1 + kCols * g + (lane - kNB);
      const bool live = c < b;
      double2 x[kNB];  // x[r] = T(k0 + r, c); rows below the diagonal start at zero
#pragma unroll
      for (int r = 0; r < kNB; ++r)
        x[r] = live && k0 + r <= c ? at(k0 + r, c) : make_double2(0.0, 0.0);
      bool bad = false;
#pragma unroll
      for (int k = 0; k < kNB; ++k) {
        double d = readlane_f64(x[k].x, k);
        bad |= !(d > 1e-300);
        d = d > 1e-300 ? d : 1e-300;
        const double ri = rsqrt(d);
        const bool piv = lane == k;
        x[k].x = piv ? d * ri : x[k].x * ri;
        x[k].y = piv ? 0.0 : x[k].y * ri;
#pragma unroll
        for (int i = k + 1; i < kNB; ++i) {
          // x_i -= conj(r_ki) x_k as four fused multiply-adds
          const double2 rki = make_double2(readlane_f64(x[k].x, i), readlane_f64(x[k].y, i));
          x[i].x = fma(-rki.x, x[k].x, fma(-rki.y, x[k].y, x[i].x));
          x[i].y = fma(-rki.x, x[k].y, fma(rki.y, x[k].x, x[i].y));
        }
      }
      if (bad && t == 0) *flag = 1;
      // diagonal of the unscaled factor (R' D^-1): converges to the
      // eigenvalue magnitudes in orthogonal iteration
      if (rdiag && g == 0 && lane < kNB) {
        double dg = 0.0;
#pragma unroll
        for (int r = 0; r < kNB; ++r) dg = r == lane ? x[r].x : dg;
        rdiag[k0 + lane] = dsc[k0 + lane] > 0.0 ? dg / dsc[k0 + lane] : 0.0;
      }
      // the diagonal block is not read again (and other groups may still be
      // loading it): its lanes write R only
      if (live && (lane >= kNB || g == 0)) {
#pragma unroll
        for (int r = 0; r < kNB; ++r)
          if (k0 + r <= c) {
            if (lane >= kNB) at(k0 + r, c) = x[r];
            R[size_t(c) * b + k0 + r] = x[r];
          }
      }
    }
    __syncthreads();
    // trailing update in 2 x 2 patches (pi <= pj) of the upper triangle,
    // patch rows below kend left to k_chol_update
    const int m = nc >> 1;
    const int mr = (kend - k1) >> 1;  // patch rows of this call
    const int npatch = m * (m + 1) / 2 - (m - mr) * (m - mr + 1) / 2;
    for (int q = t; q < npatch; q += kNT) {
      // row of patches: start(p) = p m - p (p - 1) / 2 <= q < start(p + 1)
      const double tm = 2.0 * m + 1.0;
      int pi = int((tm - sqrt(tm * tm - 8.0 * q)) * 0.5);
      pi = pi < 0 ? 0 : (pi > m - 1 ? m - 1 : pi);
      while (pi > 0 && pi * m - pi * (pi - 1) / 2 > q) --pi;
      while (pi + 1 < m && (pi + 1) * m - (pi + 1) * pi / 2 <= q) ++pi;
      const int pj = pi + q - (pi * m - pi * (pi - 1) / 2);
      const int i0 = k1 + 2 * pi, j0 = k1 + 2 * pj;
      const bool diag = pi == pj;
      double2 a00 = at(i0, j0), a01 = at(i0, j0 + 1), a11 = at(i0 + 1, j0 + 1);
      double2 a10 = diag ? make_double2(0.0, 0.0) : at(i0 + 1, j0);
#pragma unroll
      for (int l = 0; l < kNB; ++l) {
        const double2 ri0 = at(k0 + l, i0), ri1 = at(k0 + l, i0 + 1);
        const double2 rj0 = at(k0 + l, j0), rj1 = at(k0 + l, j0 + 1);
        a00 = zsub(a00, zmulc(ri0, rj0));
        a01 = zsub(a01, zmulc(ri0, rj1));
        a10 = zsub(a10, zmulc(ri1, rj0));
        a11 = zsub(a11, zmulc(ri1, rj1));
      }
      at(i0, j0) = a00;
      at(i0, j0 + 1) = a01;
      at(i0 + 1, j0 + 1) = a11;
      if (!diag) at(i0 + 1, j0) = a10;
    }
    __syncthreads();
  }
}

// Staging of the blocked Cholesky over many workgroups, one thread per
// entry (i, j) of the column-major S: the scale d_i = 1 / sqrt(S_ii) (0
// where S_ii <= 0) to dsc_out, T_ij = d_i d_j S_ij (+ shift on the diagonal,
// imaginary part dropped there) for i <= j into T (row-major, ld = b + 1),
// and zeros into R below the diagonal.
__global__ void __launch_bounds__(256) k_chol_stage(const double2* __restrict__ S, int b,
                                                    double shift, double2* __restrict__ T,
                                                    double2* __restrict__ R,
                                                    double* __restrict__ dsc_out,
                                                    const int* __restrict__ skip) {
  if (skip && *skip) return;
  const long long e = blockIdx.x * 256LL + threadIdx.x;
  if (e >= 1LL * b * b) return;
  const int i = int(e % b), j = int(e / b);
  if (j < i) {
    R[e] = make_double2(0.0, 0.0);
    return;
  }
  const double si = S[size_t(i) * b + i].x, sj = S[size_t(j) * b + j].x;
  const double di = si > 0.0 ? 1.0 / sqrt(si) : 0.0, dj = sj > 0.0 ? 1.0 / sqrt(sj) : 0.0;
  double2 v = zscale(S[e], di * dj);
  if (i == j) {
    v = make_double2(v.x + shift, 0.0);
    dsc_out[i] = di;
  }
  T[size_t(i) * (b + 1) + j] = v;
}

// Trailing update of the blocked Cholesky: T_ij -= sum_{l in [kbeg, kend)}
// conj(R_li) R_lj for kend <= i <= j < b, one 32 x 32 tile of the upper
// triangle per workgroup; the finished rows R_l,: sit in T's rows l (T
// row-major, ld = b + 1) and are staged in LDS for the tile's rows and
// columns.
constexpr int kCholPanel = 32;  // rows per panel of the blocked factorisation

__global__ void __launch_bounds__(256) k_chol_update(double2* __restrict__ T, int b, int kbeg,
                                                     int kend, const int* __restrict__ skip) {
  if (skip && *skip) return;
  __shared__ double2 Ri[kCholPanel][33], Rj[kCholPanel][33];
  const int ld = b + 1, K = kend - kbeg;
  const int nt = (b - kend + 31) / 32;
  // tile (ti, tj), ti <= tj, from the linear index (row-major upper triangle)
  const int q = blockIdx.x;
  int ti = 0;
  while ((ti + 1) * nt - (ti + 1) * ti / 2 <= q) ++ti;
  const int tj = ti + (q - (ti * nt - ti * (ti - 1) / 2));
  const int i0 = kend + 32 * ti, j0 = kend + 32 * tj;
  for (int e = threadIdx.x; e < K * 32; e += 256) {
    const int kk = e >> 5, c = e & 31;
    const size_t row = size_t(kbeg + kk) * ld;
    Ri[kk][c] = i0 + c < b ? T[row + i0 + c] : make_double2(0.0, 0.0);
    Rj[kk][c] = j0 + c < b ? T[row + j0 + c] : make_double2(0.0, 0.0);
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int e = threadIdx.x + 256 * u;
    const int ii = e >> 5, jj = e & 31;
    const int i = i0 + ii, j = j0 + jj;
    if (i >= b || j >= b || j < i) continue;
    double2 acc = make_double2(0.0, 0.0);
    for (int kk = 0; kk < K; ++kk) acc = zadd(acc, zmulc(Ri[kk][ii], Rj[kk][jj]));
    T[size_t(i) * ld + j] = zsub(T[size_t(i) * ld + j], acc);
  }
}

// M = D R^{-1}, one column j per wave: back substitution R x = e_j in
// column (axpy) order, k = j down to 0: x_k = r_k / R_kk, then
// r_i -= R_ik x_k for i < k.  Lane l holds rows l + 64 s; x_k goes from its
// owner to the wave by readlane.  Columns are independent, so the b columns
// run side by side, kTriWaves to a workgroup.  The entries of R the steps
// use are read eight steps at a time into registers, so that the chain of
// steps does not wait on memory.  With kStage the strict upper triangle of
// the columns the workgroup needs is first copied to LDS (packed, column k
// at k (k - 1) / 2); otherwise (large b) they come from global memory.
constexpr int kTriWaves = 4;
constexpr int kTriStageMax = 128;  // largest b staged in LDS

template <int kRows, bool kStage>
__global__ void __launch_bounds__(64 * kTriWaves) k_tri_inv(const double2* __restrict__ R,
                                                            const double* __restrict__ dsc,
                                                            double2* __restrict__ M, int b,
                                                            const int* __restrict__ skip) {
  if (skip && *skip) return;
  constexpr int kMaxB = 64 * kRows;  // b <= kMaxB (at most kTriStageMax when staged)
  constexpr int kStep = kRows <= 4 ? 8 : 32 / kRows;  // steps per register batch
  __shared__ double2 tri[kStage ? kMaxB * (kMaxB - 1) / 2 : 1];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int j = blockIdx.x * kTriWaves + wave;
  // the wave's own global reads first, so that their latency overlaps the
  // staging: the diagonal of R and D for rows lane + 64 s
  double rdia[kRows], dg[kRows];
#pragma unroll
  for (int s = 0; s < kRows; ++s) {
    const int i = lane + 64 * s;
    rdia[s] = i <= j && j < b ? R[size_t(i) * b + i].x : 1.0;
    dg[s] = i < b ? dsc[i] : 0.0;
  }
  if (kStage) {
    int jmax = blockIdx.x * kTriWaves + kTriWaves - 1;
    jmax = jmax < b - 1 ? jmax : b - 1;
    // wave w copies columns 1 + w, 1 + w + kTriWaves, ...; a batch of
    // columns is loaded before it is stored
    constexpr int kCols = 16;
    for (int c0 = 1 + wave; c0 <= jmax; c0 += kCols * kTriWaves) {
      double2 v[kCols][kRows];
#pragma unroll
      for (int c = 0; c < kCols; ++c) {
        const int k = c0 + c * kTriWaves;
#pragma unroll
        for (int s = 0; s < kRows; ++s) {
          const int i = lane + 64 * s;
          v[c][s] = k <= jmax && i < k ? R[size_t(k) * b + i] : make_double2(0.0, 0.0);
        }
      }
#pragma unroll
      for (int c = 0; c < kCols; ++c) {
        const int k = c0 + c * kTriWaves;
#pragma unroll
        for (int s = 0; s < kRows; ++s) {
          const int i = lane + 64 * s;
          if (k <= jmax && i < k) tri[k * (k - 1) / 2 + i] = v[c][s];
        }
      }
    }
    __syncthreads();
  }
  if (j >= b) return;
  double2 y[kRows];
  double rinv[kRows];
#pragma unroll
  for (int s = 0; s < kRows; ++s) {
    const int i = lane + 64 * s;
    y[s] = make_double2(i == j ? 1.0 : 0.0, 0.0);
    rinv[s] = 1.0 / rdia[s];
  }
  for (int kb = j; kb >= 0; kb -= kStep) {
    double2 cb[kStep][kRows];
#pragma unroll
    for (int u = 0; u < kStep; ++u) {
      const int k = kb - u;
#pragma unroll
      for (int s = 0; s < kRows; ++s) {
        const int i = lane + 64 * s;
        cb[u][s] = i < k ? (kStage ? tri[k * (k - 1) / 2 + i] : R[size_t(k) * b + i])
                         : make_double2(0.0, 0.0);
      }
    }
#pragma unroll
    for (int u = 0; u < kStep; ++u) {
      const int k = kb - u;
      if (k < 0) continue;
      const int so = k >> 6, lo = k & 63;
      double2 mine = zscale(y[0], rinv[0]);
#pragma unroll
      for (int s = 1; s < kRows; ++s)
        if (s == so) mine = zscale(y[s], rinv[s]);
      const double2 xk = make_double2(readlane_f64(mine.x, lo), readlane_f64(mine.y, lo));
#pragma unroll
      for (int s = 0; s < kRows; ++s) {
        const int i = lane + 64 * s;
        const double2 upd = zsub(y[s], zmul(cb[u][s], xk));
        // component-wise selects (a select of the pair can go through memory)
        const bool lt = i < k, eq = i == k;
        y[s].x = lt ? upd.x : (eq ? xk.x : y[s].x);
        y[s].y = lt ? upd.y : (eq ? xk.y : y[s].y);
      }
    }
  }
#pragma unroll
  for (int s = 0; s < kRows; ++s) {
    const int i = lane + 64 * s;
    if (i < b) M[size_t(j) * b + i] = i <= j ? zscale(y[s], dg[s]) : make_double2(0.0, 0.0);
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
                          int* ctl, unsigned* status, int* host_ctl,
                          const int* __restrict__ sched) {
  // one wave: the counts by ballot, the largest residual by lane shuffles
  const int t = threadIdx.x;
  const double t0 = theta[0];
  int rs = 0;
  for (int k0 = 0; k0 < b; k0 += 64) {
    const int k = k0 + t;
    rs += __popcll(__ballot(k < b && theta[k] >= thr2 * t0));
  }
  const int upto = rs + 1 < b ? rs + 1 : b;
  double worst = 0.0;
  bool bad = false;
  for (int k = t; k < upto; k += 64) {
    double s = 0.0;
    for (int c = 0; c < nchunks; ++c) s += rpart[size_t(c) * b + k];
    const double r = sqrt(s);
    bad |= !isfinite(r);
    worst = r > worst ? r : worst;
  }
  for (int off = 32; off > 0; off >>= 1) worst = fmax(worst, __shfl_xor(worst, off, 64));
  const bool finite = isfinite(t0) && __ballot(bad) == 0ull;
  if (t != 0) return;
  const int zero = !(t0 > 0.0);
  if (zero) rs = 0;
  const int too_small = rs > b - margin;
  ctl[0] = rs;
  ctl[1] = (finite && !zero && worst <= tol * t0 && !too_small) ? 1 : 0;
  ctl[2] = iter + 1 - (sched ? sched[0] : 0);  // products run (skipped slots excluded)
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
  if (host_ctl) {  // the same words, straight to pinned host memory
    for (int k = 0; k < 6; ++k) host_ctl[k] = ctl[k];
    __threadfence_system();
  }
}

// Schedule of the first Rayleigh-Ritz step and the Chebyshev filter, both
// from the Cholesky diagonal d_j after three products (d_j follows the
// eigenvalues of A on the leading columns of the block).
//
// Filter: with c = 1.05 d_{b-1}, every eigenvalue below c maps into [-1, 1]
// under x = 2 lambda / c - 1, where the Chebyshev polynomial T_j stays
// within [-1, 1], while an eigenvalue lambda_r of the signal subspace grows
// as T_j(2 lambda_r / c - 1), far faster than lambda_r^j / lambda_b^j.  A
// chain of j products then applies T_j(2A/c - I) by the three-term
// recurrence Y_1 = (2/c) A X - X, Y_{i+1} = (4/c) A Y_i - 2 Y_i - Y_{i-1}.
// coef[0..2] holds the first step, coef[3..5] the later ones; without a
// usable c (no gap, zero data) both are (1, 0, 0), plain products.
//
// Prediction: the worst residual over the signal columns, relative to
// theta_1, after a Rayleigh-Ritz step on the next product is about
// (d_{b-1} / d_0) rho^2 with rho = d_{b-1} / d_{r-1} (r the signal rank by
// the threshold); every further product divides it by the growth of its
// chain (chains of three, the remainder last, as the driver forms them) or
// by 1 / rho without the filter.  The prediction aims ten times below the
// tolerance, since a Rayleigh-Ritz step that fails costs several products.
// ctl[6] = products until (and including) the one the step is taken on.
// Device-resident schedule (plan.nslots > 0): the products between the
// third and the last one are enqueued in advance as slots in fixed chains;
// the first S = nslots - (ctl[6] - 1) slots are skipped (their product and,
// for a chain with no product left, its orthonormalisation copy the block
// instead), so that the step is taken after as many products as predicted.
// sched[0] = S, sched[1 + j] = role of slot j (0 skipped, 1 first step of
// its chain, 2 later step), sched[1 + kMaxSlots + j] = 1 when the chain
// ending at slot j is skipped entirely.
constexpr int kMaxSlots = 60;
struct SlotPlan {
  int nslots;
  signed char pos[kMaxSlots];   // position of the slot in its chain
};

__global__ void k_predict(const double* __restrict__ d, int b, double thr2, double tol, int* ctl,
                          double* __restrict__ coef, int* host_ctl, SlotPlan plan,
                          int* __restrict__ sched) {
  const int t = threadIdx.x;  // one wave: the count by ballot, the rest in lane 0
  int r = 0;
  for (int k0 = 0; k0 < b; k0 += 64) {
    const int k = k0 + t;
    r += __popcll(__ballot(k < b && d[k] >= thr2 * d[0]));
  }
  if (t != 0) return;
  const bool ok = r > 0 && r < b && d[r - 1] > 0.0 && d[b - 1] > 0.0 && isfinite(d[0]);
  const double c = 1.05 * (ok ? d[b - 1] : 0.0);
  const double x = ok ? 2.0 * d[r - 1] / c - 1.0 : 0.0;
  const bool filter = ok && x > 1.0 && isfinite(2.0 / c);
  const double f[6] = {filter ? 2.0 / c : 1.0, filter ? -1.0 : 0.0, 0.0,
                       filter ? 4.0 / c : 1.0, filter ? -2.0 : 0.0, filter ? -1.0 : 0.0};
  for (int k = 0; k < 6; ++k) coef[k] = f[k];
  int need = 4;
  if (ok) {
    double rho = d[b - 1] / d[r - 1];
    rho = rho < 1e-3 ? 1e-3 : (rho > 0.95 ? 0.95 : rho);
    const double target = log(0.1 * tol);
    const double e0 = log(d[b - 1] / d[0]) + 2.0 * log(rho);
    // log growth of chains of one, two and three filtered products
    const double g1 = filter ? log(x) : -log(rho);
    const double g2 = filter ? log(2.0 * x * x - 1.0) : -2.0 * log(rho);
    const double g3 = filter ? log((4.0 * x * x - 3.0) * x) : -3.0 * log(rho);
    need = 40;
    for (int k = 0; k < 40; ++k) {
      const int rem = k % 3;
      const double e = e0 - (k / 3) * g3 - (rem == 1 ? g1 : (rem == 2 ? g2 : 0.0));
      if (e <= target) {
        need = k + 1;
        break;
      }
    }
  }
  ctl[6] = need < 1 ? 1 : (need > 40 ? 40 : need);
  // slot 3: the coefficients of the next product, a chain's first step or a
  // plain product (1, 0, 0) when the Rayleigh-Ritz step is taken on it, so
  // that the host can enqueue it before it reads the schedule
  const bool plain = ctl[6] <= 1;
  for (int k = 0; k < 3; ++k) coef[6 + k] = plain ? (k == 0 ? 1.0 : 0.0) : f[k];
  if (sched && plan.nslots > 0) {
    int S = plan.nslots - (ctl[6] - 1);
    S = S < 0 ? 0 : (S > plan.nslots ? plan.nslots : S);
    sched[0] = S;
    for (int j = 0; j < plan.nslots; ++j) {
      sched[1 + j] = j < S ? 0 : ((plan.pos[j] == 0 || j - 1 < S) ? 1 : 2);
      sched[1 + kMaxSlots + j] = j < S ? 1 : 0;
    }
  }
  if (host_ctl) {
    host_ctl[6] = ctl[6];
    __threadfence_system();
  }
}

// Flags are raised only for a final result (converged, stopped, or at the
// product limit `max_iters`, done products so far): the adaptive schedule
// also runs this ahead of its host check and goes on when the step is not
// final.  done = max_iters = 0: always final.
__global__ void k_finalize(const double2* __restrict__ W, const double* __restrict__ theta,
                           const int* __restrict__ ctl, double2* __restrict__ basis,
                           double* __restrict__ eigvals, int32_t* __restrict__ counts,
                           long long nb, int b, int done, int max_iters, unsigned* status) {
  const long long i = blockIdx.x * 256LL + threadIdx.x;
  if (i < nb) basis[i] = W[i];
  if (i < b) eigvals[i] = theta[i];
  if (i == 0) {
    counts[0] = ctl[0];
    counts[1] = b;
    counts[2] = ctl[2];
    counts[3] = ctl[1];
    unsigned f = 0;
    const bool final = ctl[1] || ctl[3] || ctl[4] || done >= max_iters;
    if (!final) return;
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

// skip (device word, nullable): the orthonormalisation of a skipped chain
pisco_status_t gemm_tn(NullCtx& c, const double2* P, const double2* Qm, double2* out, int rows,
                       bool upper = false, const int* skip = nullptr) {
  const int b = c.b;
  const int chunks = int(ceil_div(rows, kTnRows));
  dim3 g(ceil_div(b, 16), ceil_div(b, 16), chunks);
  PISCO_KERNEL(c.h, k_gemm_tn, g, dim3(64), 0, P, Qm, c.w.part, rows, b, upper ? 1 : 0, skip);
  const long long len = 1LL * b * b;
  PISCO_KERNEL(c.h, k_sum_parts, dim3(ceil_div(len, 64)), dim3(64), 0, c.w.part, out, len, chunks,
               skip);
  return PISCO_OK;
}

pisco_status_t gemm_nn(NullCtx& c, const double2* P, const double2* M, double2* Y, int m,
                       int k, bool tri = false, const int* copy = nullptr) {
  dim3 g(ceil_div(m, 16), ceil_div(c.b, 16));
  PISCO_KERNEL(c.h, k_gemm_nn, g, dim3(64), 0, P, M, Y, m, k, c.b, tri ? 1 : 0, copy);
  return PISCO_OK;
}

pisco_status_t chol_inv(NullCtx& c, const double2* S, double shift, double2* M,
                        double* rdiag = nullptr, const int* skip = nullptr) {
  const int b = c.b;
  if (b % 8 != 0 || b > 1024) {
    c.h->last_error = "nullspace: block size must be a multiple of 8, at most 1024";
    return PISCO_ERR_UNSUPPORTED;
  }
  int* flag = c.w.ctl + 8;
  double2* T = reinterpret_cast<double2*>(c.w.jac);
  if (b <= kCholLdsMax) {
    PISCO_KERNEL(c.h, k_chol<true>, dim3(1), dim3(kCholThreads), 0, S, b, shift, c.w.R,
                 c.w.dsc, T, flag, rdiag, skip, 0, b);
  } else {
    // blocked: staged across many workgroups, then one workgroup eliminates
    // a panel of rows and many update the rest
    PISCO_KERNEL(c.h, k_chol_stage, dim3(ceil_div(1LL * b * b, 256)), dim3(256), 0, S, b, shift,
                 T, c.w.R, c.w.dsc, skip);
    for (int kb = 0; kb < b; kb += kCholPanel) {
      const int ke = kb + kCholPanel < b ? kb + kCholPanel : b;
      PISCO_KERNEL(c.h, k_chol<false>, dim3(1), dim3(kCholThreads), 0, S, b, shift, c.w.R,
                   c.w.dsc, T, flag, rdiag, skip, kb, ke);
      if (ke < b) {
        const int nt = ceil_div(b - ke, 32);
        PISCO_KERNEL(c.h, k_chol_update, dim3(nt * (nt + 1) / 2), dim3(256), 0, T, b, kb, ke,
                     skip);
      }
    }
  }
  const dim3 tg(ceil_div(b, kTriWaves)), tb(64 * kTriWaves);
  if (b <= 64)
    PISCO_KERNEL(c.h, (k_tri_inv<1, true>), tg, tb, 0, c.w.R, c.w.dsc, M, b, skip);
  else if (b <= kTriStageMax)
    PISCO_KERNEL(c.h, (k_tri_inv<2, true>), tg, tb, 0, c.w.R, c.w.dsc, M, b, skip);
  else if (b <= 256)
    PISCO_KERNEL(c.h, (k_tri_inv<4, false>), tg, tb, 0, c.w.R, c.w.dsc, M, b, skip);
  else if (b <= 384)
    PISCO_KERNEL(c.h, (k_tri_inv<6, false>), tg, tb, 0, c.w.R, c.w.dsc, M, b, skip);
  else if (b <= 512)
    PISCO_KERNEL(c.h, (k_tri_inv<8, false>), tg, tb, 0, c.w.R, c.w.dsc, M, b, skip);
  else
    PISCO_KERNEL(c.h, (k_tri_inv<16, false>), tg, tb, 0, c.w.R, c.w.dsc, M, b, skip);
  return PISCO_OK;
}

// Orthonormalise the columns of Y (n x b) by one Cholesky QR pass with
// column scaling, the result in `tmp`.  `shift` (relative to the scaled
// diagonal) keeps the factorisation from breaking down on the first
// product, whose columns may be nearly dependent; a block that is not yet
// orthonormal to rounding is fine there, the next products correct it.
// skip (device word, nullable): when set, tmp = Y.
pisco_status_t orth(NullCtx& c, const double2* Y, double2* tmp, double* rdiag, double shift,
                    const int* skip = nullptr) {
  const int n = c.p->n, b = c.b;
  pisco_status_t st;
  if ((st = gemm_tn(c, Y, Y, c.w.S, n, true, skip))) return st;  // the factor reads the upper part
  if ((st = chol_inv(c, c.w.S, shift, c.w.M, rdiag, skip))) return st;
  return gemm_nn(c, Y, c.w.M, tmp, n, b, true, skip);
}

}  // namespace

pisco_status_t run_nullspace(Handle* h, const Plan& p, int b, int max_iters,
                             const float2* gram, double* eigvals, double2* basis,
                             int32_t* counts, void* ws, int fixed_products, int ax_waves,
                             const std::function<pisco_status_t()>* downstream,
                             bool* downstream_queued, int device_products,
                             const ToeplitzOp* tp) {
  if (downstream_queued) *downstream_queued = false;
  const bool device = device_products > 0 && fixed_products <= 0;
  if (fixed_products <= 0 && !device) {
    // the adaptive schedule waits on the host for control words the kernels
    // write: it cannot be recorded into a graph
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    const hipError_t e = hipStreamIsCapturing(h->stream, &cs);
    if (e != hipSuccess) return hip_check(h, e, "nullspace capture query");
    if (cs != hipStreamCaptureStatusNone) {
      h->last_error = "the adaptive nullspace schedule reads control words on the host and "
                      "cannot be captured; use the device-resident or a fixed schedule";
      return PISCO_ERR_UNSUPPORTED;
    }
  }
  NullCtx c{h, &p, b, {}};
  layout_null(p, b, ws, &c.w, tp != nullptr);
  hipStream_t s = h->stream;
  const int n = p.n;
  const long long nb = 1LL * n * b;
  double2* W = basis;  // Ritz vectors are formed directly in the output buffer
  double2* X = c.w.X;  // current orthonormal block
  double2* Z = c.w.Z;  // A X

  // random start block; its columns need not be orthonormal, since the
  // first product is orthonormalised before any Rayleigh-Ritz step
  PISCO_KERNEL(h, k_init_block, dim3(ceil_div(nb, 256)), dim3(256), 0, X, n, b);
  pisco_status_t st = PISCO_OK;
  if (tp && (st = toeplitz_prepare(h, *tp))) return st;

  const double thr2 = double(p.thresh) * double(p.thresh);
  const double tol = 1e-10;
  const int margin = b / 8 > 4 ? b / 8 : 4;
  // K slices so that the product runs about ax_waves waves (at most kAxSplit)
  const long long tiles = 1LL * ceil_div(n, 32) * ceil_div(b, 32);
  // (a power of two: the slices of a tile form one workgroup)
  int want = int(ceil_div(ax_waves > 0 ? ax_waves : 2048, tiles));
  want = want < 1 ? 1 : (want > kAxSplit ? kAxSplit : want);
  while (want & (want - 1)) want &= want - 1;
  const int kchunk = 16 * int(ceil_div(ceil_div(n, want), 16));
  const int ksplit = want;  // slices past n (rounding) have an empty K range
  const int rchunks = int(ceil_div(n, 1024));
  // out = A in (the K slices of a tile summed in fixed order in LDS); with
  // step 1 or 2 the sum forms the first or a later step of the Chebyshev
  // recurrence instead (prev = the previous block of the chain); with a
  // role word (device-resident schedule) the step, or a copy, is decided on
  // the device from coef = the filter's six coefficients
  auto product = [&](const double2* in, double2* out, const double2* prev, int step,
                     const int* role = nullptr) -> pisco_status_t {
    const dim3 g(ceil_div(n, 32), ceil_div(b, 32));
    const double* coef = role ? c.w.filt : (step ? c.w.filt + 3 * (step - 1) : nullptr);
    if (tp) return toeplitz_product(h, *tp, in, out, n, b, coef, prev, role);
    switch (ksplit) {
      case 8:
        PISCO_KERNEL(h, k_gemm_ax<8>, g, dim3(512), 0, gram, in, out, n, b, kchunk, coef, prev,
                     role);
        break;
      case 4:
        PISCO_KERNEL(h, k_gemm_ax<4>, g, dim3(256), 0, gram, in, out, n, b, kchunk, coef, prev,
                     role);
        break;
      case 2:
        PISCO_KERNEL(h, k_gemm_ax<2>, g, dim3(128), 0, gram, in, out, n, b, kchunk, coef, prev,
                     role);
        break;
      default:
        PISCO_KERNEL(h, k_gemm_ax<1>, g, dim3(64), 0, gram, in, out, n, b, kchunk, coef, prev,
                     role);
    }
    return PISCO_OK;
  };
  // Products are counted in `done`.  Each of the first three is
  // orthonormalised on its own; the Cholesky diagonal seen after the third
  // sets the Chebyshev filter and (adaptive mode) the first Rayleigh-Ritz
  // step; later ones are scheduled from the Ritz values and residuals.
  // From then on up to three products form one filtered chain per Cholesky
  // QR pass (the scaled block stays well conditioned over such a chain).
  // The product a Rayleigh-Ritz step is taken on is a plain one.
  // With fixed_products > 0 the schedule is set in advance (that many
  // products, one Rayleigh-Ritz step at the end) and nothing is read back on
  // the host, so the whole call can be captured in a graph; the filter
  // coefficients stay on the device and convergence is still tested there,
  // reported through counts and the status.
  // The device-resident schedule enqueues the fixed schedule of
  // device_products products, and k_predict turns the leading products past
  // the third (and the orthonormalisations of chains left empty) into copies,
  // so that the Rayleigh-Ritz step follows as many products as it predicts.
  constexpr int kUnscheduled = 1 << 30;
  const bool fixed = fixed_products > 0 || device;
  const int nprod = device ? device_products : fixed_products;
  int rr_at = fixed ? (nprod < 3 ? 3 : nprod) : kUnscheduled;
  // device-resident schedule: chain position of every slot (products
  // 4 .. rr_at - 1), the structure the loop below forms for rr_at
  SlotPlan plan{};
  int* sched = device ? c.w.ctl + 16 : nullptr;
  if (device) {
    int d = 3;
    while (d + 1 < rr_at) {
      int extra = rr_at - (d + 1) - 2;
      extra = extra < 0 ? 0 : (extra > 2 ? 2 : extra);
      for (int e = 0; e <= extra; ++e) {
        if (plan.nslots >= kMaxSlots) break;
        plan.pos[plan.nslots++] = static_cast<signed char>(e);
      }
      d += extra + 1;
    }
  }
  int done = 0;
  bool filtered = false;  // filter coefficients set
  bool queued = false;    // the next product is already enqueued
  while (true) {
    const bool rr_next = done + 1 >= rr_at || done + 1 >= max_iters;
    const bool chain = filtered && !rr_next;
    // slot of the device-resident schedule this product fills (-1: none)
    const int slot = device && filtered && !rr_next ? done - 3 : -1;
    if (!queued &&
        (st = product(X, Z, nullptr, chain ? 1 : 0, slot >= 0 ? sched + 1 + slot : nullptr)))
      return st;
    queued = false;
    ++done;
    if (done < rr_at && done < max_iters) {
      int extra = 0;
      if (done > 3 && rr_at != kUnscheduled) {
        // in the fixed schedule the last orthonormalisation before the single
        // Rayleigh-Ritz step follows one product only (best conditioned)
        extra = rr_at - done - (fixed ? 2 : 1);
        extra = extra < 0 ? 0 : (extra > 2 ? 2 : extra);
      }
      for (int e = 0; e < extra; ++e) {
        // next block of the chain, written over the previous one (in X)
        const int sl = device ? done - 3 : -1;
        if ((st = chain ? product(Z, X, X, 2, sl >= 0 ? sched + 1 + sl : nullptr)
                        : product(Z, X, nullptr, 0)))
          return st;
        std::swap(X, Z);
        ++done;
      }
      const bool at3 = done == 3 && !filtered;
      // the chain just formed ended at slot done - 4
      const int* skip = device && done > 3 ? sched + 1 + kMaxSlots + (done - 4) : nullptr;
      if ((st = orth(c, Z, X, at3 ? c.w.resid : nullptr, done == 1 ? 1e-12 : 0.0, skip)))
        return st;
      if (at3) {
        PISCO_KERNEL(h, k_predict, dim3(1), dim3(64), 0, c.w.resid, b, thr2, tol, c.w.ctl,
                     c.w.filt, fixed ? nullptr : h->host_ctl_dev, plan, sched);
        filtered = true;
        if (!fixed) {
          // whatever the schedule, a product comes next: enqueued now with
          // the coefficients k_predict leaves in slot 3 (plain when the
          // iteration limit makes it the last), so that it runs while the
          // host waits (on an event, for k_predict alone) for the schedule
          hipError_t e = hipSuccess;
          if (!h->sched_ev) e = hipEventCreateWithFlags(&h->sched_ev, hipEventDisableTiming);
          if (e == hipSuccess) e = hipEventRecord(h->sched_ev, s);
          if (e != hipSuccess) return hip_check(h, e, "nullspace schedule event");
          if ((st = product(X, Z, nullptr, done + 1 >= max_iters ? 0 : 3))) return st;
          queued = true;
          e = hipEventSynchronize(h->sched_ev);
          if (e != hipSuccess) return hip_check(h, e, "nullspace predict");
          rr_at = done + reinterpret_cast<volatile int*>(h->host_ctl)[6];
        }
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
                 margin, done - 1, c.w.ctl, h->status_dev, fixed ? nullptr : h->host_ctl_dev,
                 sched);
    if (fixed) break;
    // Most steps are final: k_finalize and the caller's later stages go in
    // now and the host waits (on an event) for k_control alone.  When the
    // step is not final the iteration goes on; those results are then
    // overwritten after a later step (k_finalize raises flags only for a
    // final result, and the later stages do not touch this workspace).
    hipError_t e = hipSuccess;
    if (!h->sched_ev) e = hipEventCreateWithFlags(&h->sched_ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(h->sched_ev, s);
    if (e != hipSuccess) return hip_check(h, e, "nullspace schedule event");
    PISCO_KERNEL(h, k_finalize, dim3(ceil_div(nb > b ? nb : b, 256)), dim3(256), 0, W,
                 c.w.theta, c.w.ctl, basis, eigvals, counts, nb, b, done, max_iters,
                 h->status_dev);
    if (downstream && *downstream) {
      if ((st = (*downstream)())) return st;
      if (downstream_queued) *downstream_queued = true;
    }
    e = hipEventSynchronize(h->sched_ev);
    if (e != hipSuccess) return hip_check(h, e, "nullspace sync");
    const volatile int* hc = h->host_ctl;
    if (hc[1] || hc[3] || hc[4] || done >= max_iters) return PISCO_OK;
    if (downstream_queued) *downstream_queued = false;
    rr_at = done + hc[5];
    // next block: orth(A * Ritz vectors) (held in X; nearly orthogonal columns)
    if ((st = orth(c, X, Z, nullptr, 0.0))) return st;
    std::swap(X, Z);
  }
  PISCO_KERNEL(h, k_finalize, dim3(ceil_div(nb > b ? nb : b, 256)), dim3(256), 0, W,
               c.w.theta, c.w.ctl, basis, eigvals, counts, nb, b, 0, 0, h->status_dev);
  return PISCO_OK;
}

}  // namespace pisco
