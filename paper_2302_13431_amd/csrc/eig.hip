// Per-voxel eigenvector of G(x) for its smallest eigenvalue by power
// iteration (Sec. III-D step 4, Sec. IV-E), with an optional FP64 Rayleigh
// check of the result.
//
// Power iteration finds the dominant eigenvector, so it runs on
// Gs(x) = |Lambda| I - G(x), whose spectrum is |Lambda| minus that of G
// (0 <= G <= |Lambda| I because G = Phi^H conj(W) Phi with W a projector and
// Phi^H Phi = |Lambda| I); the top eigenvector of Gs is the bottom one of G.
//
// The start vector is e_q* (q* = argmin_q G_qq, lowest q on ties) or, when
// given, the caller's per-voxel vector (a warm start, normalised here).
//
// Mapping: a wave holds 64 / QG voxels, QG = the next power of two >= Q
// lanes each; lane q of a voxel holds row q of Gs in registers and
// component q of the iterate.  A workgroup of four waves first stages its
// voxels' G in LDS: G is stored entry-major ([pair][voxel]), so each packed
// plane contributes one contiguous run of the workgroup's voxels, loaded by
// coalesced reads.  After that one barrier every wave runs on its own: the
// iterate goes through a wave-private LDS slot, read as broadcasts for the
// product, and norms, Rayleigh quotients and residuals are xor-butterfly
// sums over the voxel's lanes.  Such a sum leaves the bitwise same value in
// every lane (IEEE addition commutes), so the lanes of a voxel take the same
// decisions (start index, convergence).  A wave leaves as soon as all of its
// voxels are done.
#include "common.hpp"

namespace pisco {

__device__ inline int pidx(int p, int q, int Q) {  // p <= q
  return p * Q - p * (p - 1) / 2 + (q - p);
}

// xor-butterfly sum over the QG lanes of a voxel (the same bits in every lane)
template <int QG, class T>
__device__ inline T vsum(T x) {
#pragma unroll
  for (int m = 1; m < QG; m <<= 1) x += __shfl_xor(x, m, QG);
  return x;
}

// two such sums at once (independent shuffles interleaved)
template <int QG>
__device__ inline void vsum2(float& a, float& b) {
#pragma unroll
  for (int m = 1; m < QG; m <<= 1) {
    const float oa = __shfl_xor(a, m, QG), ob = __shfl_xor(b, m, QG);
    a += oa;
    b += ob;
  }
}

template <int QG>
__global__ void __launch_bounds__(256, 3) k_power(const float2* __restrict__ G, int Q, long long N,
                                               float bound, int iters, float tol,
                                               const float2* __restrict__ init,
                                               float2* __restrict__ maps,
                                               float* __restrict__ lam,
                                               int32_t* __restrict__ itout,
                                               double* __restrict__ lam64,
                                               double* __restrict__ res64, unsigned* status) {
  constexpr int VW = 64 / QG;              // voxels per wave
  constexpr int VB = 4 * VW;               // voxels per workgroup
  constexpr int PS = VB + 1;               // padded plane row in LDS
  constexpr int PM = QG * (QG + 1) / 2;    // planes at most
  __shared__ float2 gt[PM * PS];
  __shared__ float2 xw[4][64];             // per wave: the iterate, lane-indexed
  const int t = threadIdx.x, wv = t >> 6, l = t & 63;
  const int q = l % QG, slot = l / QG;
  const int P = Q * (Q + 1) / 2;
  // XCD-contiguous voxel blocks: a block's plane runs share 128-byte lines
  // with its neighbours', fetched once into one L2
  const long long v0 = xcd_block(blockIdx.x, gridDim.x) * VB;
  {
    // eight loads per thread in flight at once
    constexpr int kU = 8;
    for (int e0 = t; e0 < P * VB; e0 += 256 * kU) {
      float2 g[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int e = e0 + 256 * u, pl = e / VB, vx = e - pl * VB;
        g[u] = e < P * VB && v0 + vx < N ? G[size_t(pl) * N + v0 + vx] : make_float2(0.f, 0.f);
      }
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int e = e0 + 256 * u, pl = e / VB, vx = e - pl * VB;
        if (e < P * VB) gt[pl * PS + vx] = g[u];
      }
    }
  }
  __syncthreads();
  const int vx = wv * VW + slot;
  const bool valid = v0 + vx < N;
  const long long v = valid ? v0 + vx : N - 1;  // clamped: every load is in bounds
  const bool row = q < Q;
  // row q of Gs = bound I - G (the FP64 check re-reads G from LDS, since
  // bound - g is not exact in FP32)
  float2 gs[QG];
  float gqq = 0.f;
  bool bad = false;
#pragma unroll
  for (int p = 0; p < QG; ++p) {
    float2 g = make_float2(0.f, 0.f);
    if (row && p < Q) {
      g = q <= p ? gt[pidx(q, p, Q) * PS + vx] : cconj(gt[pidx(p, q, Q) * PS + vx]);
      bad |= !isfinite(g.x) || !isfinite(g.y);
    }
    if (p == q) gqq = g.x;
    gs[p] = p == q ? make_float2(bound - g.x, 0.f) : make_float2(-g.x, -g.y);
  }
  if (bad && valid) atomicOr(status, PISCO_FLAG_NONFINITE);
  // start vector: e_q* (q* = argmax_q Gs_qq, lowest q on ties), replaced by
  // the caller's vector when that is nonzero and finite
  float bd = row ? bound - gqq : -INFINITY;
  int bi = q;
#pragma unroll
  for (int m = 1; m < QG; m <<= 1) {
    const float od = __shfl_xor(bd, m, QG);
    const int oi = __shfl_xor(bi, m, QG);
    if (od > bd || (od == bd && oi < bi)) {
      bd = od;
      bi = oi;
    }
  }
  // iterate x = xr * xsc: xr the last product (unnormalised), xsc 1 / ||xr||
  float2 xr = make_float2(row && q == bi ? 1.f : 0.f, 0.f);
  float xsc = 1.f;
  if (init) {
    const float2 s = row ? init[size_t(q) * N + v] : make_float2(0.f, 0.f);
    const float nn = vsum<QG>(fmaf(s.x, s.x, s.y * s.y));
    if (nn > 0.f && isfinite(nn)) {
      const float inv = rsqrtf(nn);
      xr = make_float2(s.x * inv, s.y * inv);
    }
  }
  float2* xv = &xw[wv][slot * QG];
  // y = Gs x for this lane's row
  auto product = [&](float2 xq, float scale) {
    wave_sync();
    xw[wv][l] = xq;
    wave_sync();
    float2 y = make_float2(0.f, 0.f);
#pragma unroll
    for (int p = 0; p < QG; ++p) {
      const float2 x = xv[p];
      y.x = fmaf(gs[p].x, x.x, fmaf(-gs[p].y, x.y, y.x));
      y.y = fmaf(gs[p].x, x.y, fmaf(gs[p].y, x.x, y.y));
    }
    return make_float2(y.x * scale, y.y * scale);
  };
  int steps = 0;
  bool done = false;
  const float stop = tol * bound;
  for (int it = 0; it < iters; ++it) {
    const float2 y = product(xr, xsc);  // Gs x
    if (!done) {
      // ||Gs x||^2, and for the residual of the iterate the Rayleigh
      // quotient mu; ||Gs x - mu x|| = ||G x - lambda x||
      const float2 x = make_float2(xr.x * xsc, xr.y * xsc);
      float nn = fmaf(y.x, y.x, y.y * y.y), mu = fmaf(x.x, y.x, x.y * y.y);
      if (tol > 0.f) {
        vsum2<QG>(nn, mu);
        const float rx = y.x - mu * x.x, ry = y.y - mu * x.y;
        done = sqrtf(vsum<QG>(fmaf(rx, rx, ry * ry))) <= stop;
      } else {
        nn = vsum<QG>(nn);
      }
      if (!done) {
        const float nrm = sqrtf(nn);
        xsc = nrm > 0.f ? 1.f / nrm : 0.f;
        xr = y;
        ++steps;
      }
    }
    // every voxel of the wave converged: the wave leaves
    if (tol > 0.f && __all(done || !valid)) break;
  }
  const float2 c = make_float2(xr.x * xsc, xr.y * xsc);
  const float2 y = product(xr, xsc);
  const float mu = vsum<QG>(fmaf(c.x, y.x, c.y * y.y));
  if (row && valid) maps[size_t(q) * N + v] = c;
  if (q == 0 && valid) {
    if (lam) lam[v] = bound - mu;
    if (itout) itout[v] = steps;
  }
  if (lam64 || res64) {
    // G c in FP64 on the FP32 result c (widened) with G widened exactly (the
    // staged entries, diagonal real)
    wave_sync();
    xw[wv][l] = c;
    wave_sync();
    double yr = 0.0, yi = 0.0;
    for (int p = 0; p < Q && row; ++p) {
      const float2 xp = xv[p];
      float2 g = q <= p ? gt[pidx(q, p, Q) * PS + vx] : cconj(gt[pidx(p, q, Q) * PS + vx]);
      if (p == q) g.y = 0.f;
      const double cr = double(xp.x), ci = double(xp.y), gr = double(g.x), gi = double(g.y);
      yr = fma(gr, cr, fma(-gi, ci, yr));
      yi = fma(gr, ci, fma(gi, cr, yi));
    }
    // c normalised in FP64; lambda = c^H G c, residual ||G c - lambda c||
    const double cr = double(c.x), ci = double(c.y);
    const double ss = vsum<QG>(fma(cr, cr, ci * ci));
    const double num = vsum<QG>(fma(cr, yr, ci * yi));
    const double l64 = ss > 0.0 ? num / ss : 0.0;
    const double rx = yr - l64 * cr, ry = yi - l64 * ci;
    const double r2 = vsum<QG>(fma(rx, rx, ry * ry));
    if (q == 0 && valid) {
      if (lam64) lam64[v] = l64;
      if (res64) res64[v] = ss > 0.0 ? sqrt(r2 / ss) : 0.0;
    }
  }
}

pisco_status_t run_eig(Handle* h, int Q, long long N, float bound, int iters, float tol,
                       const float2* G, const float2* init, float2* maps, float* lam,
                       int32_t* it_out, double* lam64, double* res64) {
  if (N <= 0) return PISCO_OK;
#define PISCO_POWER(QG)                                                                         \
  PISCO_KERNEL(h, (k_power<QG>), dim3(ceil_div(N, 4 * (64 / QG))), dim3(256), 0, G, Q, N, bound, \
               iters, tol, init, maps, lam, it_out, lam64, res64, h->status_dev)
  if (Q <= 2) PISCO_POWER(2);
  else if (Q <= 4) PISCO_POWER(4);
  else if (Q <= 8) PISCO_POWER(8);
  else if (Q <= 16) PISCO_POWER(16);
  else PISCO_POWER(32);
#undef PISCO_POWER
  return PISCO_OK;
}

}  // namespace pisco
