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
// Mapping: a workgroup takes VPW voxels (16 or 32) and one thread per
// (row q, voxel): thread t holds row q = t / VPW of Gs for voxel t % VPW in
// registers.  G is stored entry-major ([pair][voxel]), so for every entry a
// load instruction reads VPW consecutive voxels of one plane (64 / VPW
// planes per wave): whole 128- or 256-byte segments.  Each step writes the rows of
// the product y = Gs x to LDS; after one barrier every thread reads its
// voxel's whole y (norm, residual) and the next step reads it as the
// iterate, scaled by 1 / ||y||.  y is double-buffered, so one barrier per
// step suffices.  Decisions (start index, convergence) are taken by every
// thread of a voxel from the same LDS values in the same order, so they
// agree without further synchronisation.
#include "common.hpp"

namespace pisco {

__device__ inline int pidx(int p, int q, int Q) {  // p <= q
  return p * Q - p * (p - 1) / 2 + (q - p);
}

template <int QM, int VPW>
__global__ void __launch_bounds__(QM * VPW) k_power(const float2* __restrict__ G, int Q,
                                                long long N, float bound, int iters, float tol,
                                                const float2* __restrict__ init,
                                                float2* __restrict__ maps,
                                                float* __restrict__ lam,
                                                int32_t* __restrict__ itout,
                                                double* __restrict__ lam64,
                                                double* __restrict__ res64,
                                                unsigned* status) {
  // ys[buf][p][voxel]: the product of the step (unnormalised)
  __shared__ float2 ys[2][QM][VPW];
  __shared__ double2 y64[QM][VPW];
  __shared__ float dg[QM][VPW];
  const int t = threadIdx.x;
  const int vl = t % VPW, q = t / VPW;
  const long long v0 = 1LL * blockIdx.x * VPW;
  const long long vraw = v0 + vl;
  const bool valid = vraw < N;
  const long long v = valid ? vraw : N - 1;  // clamped: every load is in bounds
  const bool row = q < Q;
  // row q of Gs = bound I - G (registers); the raw diagonal entry is kept
  // for the FP64 check, since bound - g is not exact in FP32
  float2 gs[QM];
  float gqq = 0.f;
  bool bad = false;
#pragma unroll
  for (int p = 0; p < QM; ++p) {
    float2 g = make_float2(0.f, 0.f);
    if (row && p < Q) {
      g = q <= p ? G[size_t(pidx(q, p, Q)) * N + v] : cconj(G[size_t(pidx(p, q, Q)) * N + v]);
      bad |= !isfinite(g.x) || !isfinite(g.y);
    }
    const bool on_diag = p == q;
    if (on_diag) gqq = g.x;
    gs[p] = on_diag ? make_float2(bound - g.x, 0.f) : make_float2(-g.x, -g.y);
  }
  if (bad && valid) atomicOr(status, PISCO_FLAG_NONFINITE);
  // start vector: e_q* (q* = argmax_q Gs_qq, lowest q on ties), replaced by
  // the caller's vector when that is nonzero and finite; written to ys[1]
  // as the "previous product" of step 0 with unit norm
  if (row) dg[q][vl] = bound - gqq;
  __syncthreads();
  int qs = 0;
  {
    float best = dg[0][vl];
    for (int p = 1; p < Q; ++p) {
      const float d = dg[p][vl];
      if (d > best) {
        best = d;
        qs = p;
      }
    }
  }
  float2 x0 = make_float2(q == qs ? 1.f : 0.f, 0.f);
  if (init) {
    float nn = 0.f;
    for (int p = 0; p < Q; ++p) {
      const float2 s = init[size_t(p) * N + v];
      nn = fmaf(s.x, s.x, fmaf(s.y, s.y, nn));
    }
    if (nn > 0.f && isfinite(nn)) {
      const float inv = rsqrtf(nn);
      const float2 s = row ? init[size_t(q) * N + v] : make_float2(0.f, 0.f);
      x0 = make_float2(s.x * inv, s.y * inv);
    }
  }
  if (row) ys[1][q][vl] = x0;
  __syncthreads();
  // per voxel: the iterate is x = ys[bx] * xs (xs = 1 / ||ys[bx]||); a step
  // writes the product Gs x into ys[bx ^ 1].  A converged voxel keeps bx
  // and xs and rewrites the same product each later step (bitwise the same
  // values, so a sibling still reading that slot is not disturbed)
  int bx = 1, steps = 0;
  float xs = 1.f;
  bool done = false;
  const float stop = tol * bound;
  for (int it = 0; it < iters; ++it) {
    const int wr = bx ^ 1;
    float2 y = make_float2(0.f, 0.f);
#pragma unroll
    for (int p = 0; p < QM; ++p) {
      if (p < Q) {
        const float2 x = ys[bx][p][vl];
        y.x = fmaf(gs[p].x, x.x, fmaf(-gs[p].y, x.y, y.x));
        y.y = fmaf(gs[p].x, x.y, fmaf(gs[p].y, x.x, y.y));
      }
    }
    if (row) ys[wr][q][vl] = make_float2(y.x * xs, y.y * xs);
    __syncthreads();
    if (!done) {
      if (tol > 0.f) {
        // residual of the iterate x: ||Gs x - mu x|| = ||G x - lambda x||
        float mu = 0.f;
        for (int p = 0; p < Q; ++p) {
          const float2 yp = ys[wr][p][vl], xp = ys[bx][p][vl];
          mu = fmaf(xp.x * xs, yp.x, fmaf(xp.y * xs, yp.y, mu));
        }
        float r2 = 0.f;
        for (int p = 0; p < Q; ++p) {
          const float2 yp = ys[wr][p][vl], xp = ys[bx][p][vl];
          const float rx = yp.x - mu * (xp.x * xs), ry = yp.y - mu * (xp.y * xs);
          r2 = fmaf(rx, rx, fmaf(ry, ry, r2));
        }
        done = sqrtf(r2) <= stop;
      }
      if (!done) {
        float nn = 0.f;
        for (int p = 0; p < Q; ++p) {
          const float2 yp = ys[wr][p][vl];
          nn = fmaf(yp.x, yp.x, fmaf(yp.y, yp.y, nn));
        }
        const float nrm = sqrtf(nn);
        xs = nrm > 0.f ? 1.f / nrm : 0.f;
        bx = wr;
        ++steps;
      }
    }
    // every voxel of the workgroup converged (each thread of a voxel took
    // the same decision from the same values): all leave together
    if (tol > 0.f && __syncthreads_and(done || !valid)) break;
  }
  __syncthreads();
  // lambda_min = bound - x^H Gs x; the product goes to ys[bx ^ 1] (no
  // thread reads that slot now)
  {
    float2 y = make_float2(0.f, 0.f);
#pragma unroll
    for (int p = 0; p < QM; ++p) {
      if (p < Q) {
        const float2 xp = ys[bx][p][vl];
        const float2 x = make_float2(xp.x * xs, xp.y * xs);
        y.x = fmaf(gs[p].x, x.x, fmaf(-gs[p].y, x.y, y.x));
        y.y = fmaf(gs[p].x, x.y, fmaf(gs[p].y, x.x, y.y));
      }
    }
    if (row) ys[bx ^ 1][q][vl] = y;
  }
  if (row && valid) {
    const float2 xq = ys[bx][q][vl];
    maps[size_t(q) * N + v] = make_float2(xq.x * xs, xq.y * xs);
  }
  const bool check = lam64 || res64;
  if (check && row) {
    // y64 = G c in FP64 on the FP32 result c (the stored map, widened) with
    // G widened exactly (off-diagonal -Gs, diagonal the raw entry)
    double yr = 0.0, yi = 0.0;
#pragma unroll
    for (int p = 0; p < QM; ++p) {
      if (p < Q) {
        const float2 xp = ys[bx][p][vl];
        const double cr = double(xp.x * xs), ci = double(xp.y * xs);
        const double gr = p == q ? double(gqq) : -double(gs[p].x);
        const double gi = p == q ? 0.0 : -double(gs[p].y);
        yr = fma(gr, cr, fma(-gi, ci, yr));
        yi = fma(gr, ci, fma(gi, cr, yi));
      }
    }
    y64[q][vl] = make_double2(yr, yi);
  }
  __syncthreads();
  if (q == 0 && valid) {
    float mu = 0.f;
    for (int p = 0; p < Q; ++p) {
      const float2 xp = ys[bx][p][vl], yp = ys[bx ^ 1][p][vl];
      mu = fmaf(xp.x * xs, yp.x, fmaf(xp.y * xs, yp.y, mu));
    }
    if (lam) lam[v] = bound - mu;
    if (itout) itout[v] = steps;
    if (check) {
      // c normalised in FP64; lambda = c^H G c, residual ||G c - lambda c||
      double ss = 0.0, num = 0.0;
      for (int p = 0; p < Q; ++p) {
        const float2 xp = ys[bx][p][vl];
        const double cr = double(xp.x * xs), ci = double(xp.y * xs);
        const double2 yp = y64[p][vl];
        ss = fma(cr, cr, fma(ci, ci, ss));
        num = fma(cr, yp.x, fma(ci, yp.y, num));
      }
      const double l = ss > 0.0 ? num / ss : 0.0;
      double r2 = 0.0;
      for (int p = 0; p < Q; ++p) {
        const float2 xp = ys[bx][p][vl];
        const double cr = double(xp.x * xs), ci = double(xp.y * xs);
        const double2 yp = y64[p][vl];
        const double rx = yp.x - l * cr, ry = yp.y - l * ci;
        r2 = fma(rx, rx, fma(ry, ry, r2));
      }
      if (lam64) lam64[v] = l;
      if (res64) res64[v] = ss > 0.0 ? sqrt(r2 / ss) : 0.0;
    }
  }
}

pisco_status_t run_eig(Handle* h, int Q, long long N, float bound, int iters, float tol,
                       const float2* G, const float2* init, float2* maps, float* lam,
                       int32_t* it_out, double* lam64, double* res64) {
  if (N <= 0) return PISCO_OK;
  // 32 voxels per workgroup (256-byte segments per plane) unless that leaves
  // fewer than 256 workgroups; 16 (128-byte segments) for Q > 16, where 32
  // rows of 32 voxels would leave a thread too few registers for its row
  const bool wide = N >= 256LL * 32;
  const int rows = (Q + 1) / 2 * 2;
#define PISCO_POWER(QM, VPW)                                                                    \
  PISCO_KERNEL(h, (k_power<QM, VPW>), dim3(ceil_div(N, VPW)), dim3(VPW * rows), 0, G, Q, N,    \
               bound, iters, tol, init, maps, lam, it_out, lam64, res64, h->status_dev)
  if (Q <= 8) {
    if (wide) PISCO_POWER(8, 32); else PISCO_POWER(8, 16);
  } else if (Q <= 16) {
    if (wide) PISCO_POWER(16, 32); else PISCO_POWER(16, 16);
  } else {
    PISCO_POWER(32, 16);
  }
#undef PISCO_POWER
  return PISCO_OK;
}

}  // namespace pisco
