// Per-voxel eigenvector of G(x) for its smallest eigenvalue by power
// iteration (Sec. III-D step 4, Sec. IV-E).
//
// Power iteration finds the dominant eigenvector, so it runs on
// Gs(x) = |Lambda| I - G(x), whose spectrum is |Lambda| minus that of G
// (0 <= G <= |Lambda| I because G = Phi^H conj(W) Phi with W a projector and
// Phi^H Phi = |Lambda| I); the top eigenvector of Gs is the bottom one of G.
//
// The start vector is e_q* (q* = argmin_q G_qq) or, when given, the caller's
// per-voxel vector (a warm start, normalised here).
//
// Mapping: one voxel per group of QG = next_pow2(Q) lanes; lane q holds row q
// of Gs in registers and component q of the iterate.  The matrix-vector
// product gathers the iterate with cross-lane shuffles inside the group and
// the norms are butterfly reductions, so a step touches no memory.
#include "common.hpp"

namespace pisco {

__device__ inline int pidx(int p, int q, int Q) {  // p <= q
  return p * Q - p * (p - 1) / 2 + (q - p);
}

template <int QG>
__device__ inline float group_sum(float v) {
#pragma unroll
  for (int off = QG / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, QG);
  return v;
}

template <int QG>
__global__ void __launch_bounds__(256) k_power(const float2* __restrict__ G, int Q,
                                               long long N, float bound, int iters, float tol,
                                               const float2* __restrict__ init,
                                               float2* __restrict__ maps,
                                               float* __restrict__ lam,
                                               int32_t* __restrict__ itout,
                                               unsigned* status) {
  const int lane = threadIdx.x % QG;
  const long long v = blockIdx.x * (256LL / QG) + threadIdx.x / QG;
  const bool valid = v < N;
  const bool row = valid && lane < Q;
  // row `lane` of Gs = bound I - G
  float2 gs[QG];
  bool bad = false;
  float diag = -3.0e38f;
#pragma unroll
  for (int p = 0; p < QG; ++p) {
    float2 g = make_float2(0.f, 0.f);
    if (row && p < Q) {
      g = lane <= p ? G[size_t(pidx(lane, p, Q)) * N + v]
                    : cconj(G[size_t(pidx(p, lane, Q)) * N + v]);
      bad |= !isfinite(g.x) || !isfinite(g.y);
    }
    const bool on_diag = p == lane && row;
    gs[p] = on_diag ? make_float2(bound - g.x, 0.f) : make_float2(-g.x, -g.y);
    if (on_diag) diag = bound - g.x;
  }
  if (bad) atomicOr(status, PISCO_FLAG_NONFINITE);
  // start vector e_q*, q* = argmin_q G_qq = argmax_q Gs_qq (lowest q on ties)
  float best = diag;
  int bidx = row ? lane : QG;
#pragma unroll
  for (int off = QG / 2; off > 0; off >>= 1) {
    const float ob = __shfl_xor(best, off, QG);
    const int oi = __shfl_xor(bidx, off, QG);
    if (ob > best || (ob == best && oi < bidx)) {
      best = ob;
      bidx = oi;
    }
  }
  float2 x = make_float2(lane == bidx ? 1.f : 0.f, 0.f);
  if (init) {
    // caller's start vector (a warm start); e_q* stays the fallback when it
    // is zero or not finite
    const float2 s0 = row ? init[size_t(lane) * N + v] : make_float2(0.f, 0.f);
    const float nn = group_sum<QG>(s0.x * s0.x + s0.y * s0.y);
    if (nn > 0.f && isfinite(nn)) {
      const float inv = rsqrtf(nn);
      x = make_float2(s0.x * inv, s0.y * inv);
    }
  }
  int done = 0, steps = 0;
  const float stop = tol * bound;
  const int cap = iters;
  for (int it = 0; it < cap; ++it) {
    // y = Gs x
    float2 y = make_float2(0.f, 0.f);
#pragma unroll
    for (int p = 0; p < QG; ++p) {
      const float xr = __shfl(x.x, p, QG), xi = __shfl(x.y, p, QG);
      y.x = fmaf(gs[p].x, xr, fmaf(-gs[p].y, xi, y.x));
      y.y = fmaf(gs[p].x, xi, fmaf(gs[p].y, xr, y.y));
    }
    if (tol > 0.f) {
      // residual of the current iterate: ||Gs x - mu x|| = ||G x - lambda x||
      const float mu = group_sum<QG>(x.x * y.x + x.y * y.y);
      const float rx = y.x - mu * x.x, ry = y.y - mu * x.y;
      const float r = sqrtf(group_sum<QG>(rx * rx + ry * ry));
      done = r <= stop;
    }
    if (done) break;  // uniform within the group
    const float nrm = sqrtf(group_sum<QG>(y.x * y.x + y.y * y.y));
    const float inv = nrm > 0.f ? 1.f / nrm : 0.f;
    x = make_float2(y.x * inv, y.y * inv);
    ++steps;
  }
  // lambda_min = c^H G c = bound - c^H Gs c
  float2 y = make_float2(0.f, 0.f);
#pragma unroll
  for (int p = 0; p < QG; ++p) {
    const float xr = __shfl(x.x, p, QG), xi = __shfl(x.y, p, QG);
    y.x = fmaf(gs[p].x, xr, fmaf(-gs[p].y, xi, y.x));
    y.y = fmaf(gs[p].x, xi, fmaf(gs[p].y, xr, y.y));
  }
  const float mu = group_sum<QG>(x.x * y.x + x.y * y.y);
  if (row) maps[size_t(lane) * N + v] = x;
  if (valid && lane == 0) {
    if (lam) lam[v] = bound - mu;
    if (itout) itout[v] = steps;
  }
}

pisco_status_t run_eig(Handle* h, int Q, long long N, float bound, int iters, float tol,
                       const float2* G, const float2* init, float2* maps, float* lam,
                       int32_t* it_out) {
  if (N <= 0) return PISCO_OK;
#define PISCO_POWER(QG)                                                                \
  PISCO_KERNEL(h, k_power<QG>, dim3(ceil_div(N, 256 / QG)), dim3(256), 0, G, Q, N, bound, \
               iters, tol, init, maps, lam, it_out, h->status_dev)
  if (Q <= 4)
    PISCO_POWER(4);
  else if (Q <= 8)
    PISCO_POWER(8);
  else if (Q <= 16)
    PISCO_POWER(16);
  else
    PISCO_POWER(32);
#undef PISCO_POWER
  return PISCO_OK;
}

}  // namespace pisco
