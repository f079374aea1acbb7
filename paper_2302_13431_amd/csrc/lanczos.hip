// Per-voxel Lanczos solver: the M smallest eigenpairs of G(x) (Sec. IV-E,
// Sec. III-B).
//
// Power iteration converges at the rate (|Lambda| - lambda_2)/(|Lambda| -
// lambda_1) of the shifted matrix, slowly where the two smallest eigenvalues
// of G(x) (the two smallest singular values of H(x)) are close; the paper
// names Lanczos-type methods as the remedy there.  When the field of view is
// too small for the object (aliasing, the footnote of Sec. III-B), G(x) has
// several eigenvalues near zero and one map per small eigenvalue is kept
// (multiple sets of maps).  This solver gives both: K Lanczos steps on G(x)
// from e_q* (q* = argmin_q G_qq) with full reorthogonalisation (classical
// Gram-Schmidt, twice), the tridiagonal T = V^H G V eigen-decomposed in FP64
// (bisection on Sturm counts, twisted factorisation), and the Ritz vectors
// of the M smallest Ritz values.  With K = Q the Krylov basis spans the
// whole space and the pairs are G's own to rounding.  A step whose new
// vector vanishes (an invariant subspace; also the breakdown at the end of a
// smaller Krylov space) continues from the next unit vector orthogonalised
// against the basis, with a zero coupling in T.
//
// Mapping: one voxel per group of QG = next_pow2(Q) lanes; lane q holds row q
// of G(x) in registers and component q of every vector; products gather the
// vector with cross-lane shuffles and inner products are butterfly sums
// within the group.  The Lanczos vectors live in LDS; the small tridiagonal
// problem is solved by the group's first lane.
#include <cfloat>

#include "common.hpp"
#include "tridiag.hpp"

namespace pisco {

namespace {

__device__ inline int lz_pidx(int p, int q, int Q) {  // p <= q
  return p * Q - p * (p - 1) / 2 + (q - p);
}

template <int QG>
__device__ inline float lz_sum(float v) {
#pragma unroll
  for (int off = QG / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, QG);
  return v;
}

constexpr int kMaxSets = 8;

template <int QG>
__global__ void __launch_bounds__(256) k_lanczos(const float2* __restrict__ G, int Q, long long N,
                                                 float bound, int K, int M,
                                                 float2* __restrict__ maps,
                                                 float* __restrict__ lam,
                                                 float* __restrict__ resid, unsigned* status) {
  constexpr int NG = 256 / QG;  // voxel groups per workgroup
  __shared__ float2 Vs[NG][QG][QG];     // [group][vector][component]
  __shared__ double td[NG][QG], te[NG][QG], te2[NG][QG], tw[NG][2][QG], tz[NG][QG];
  __shared__ double th[NG][kMaxSets];
  const int lane = threadIdx.x % QG, grp = threadIdx.x / QG;
  const long long vraw = blockIdx.x * (long long)NG + grp;
  const bool valid = vraw < N;
  const long long v = valid ? vraw : N - 1;
  const bool row = lane < Q;
  // row `lane` of G
  float2 g[QG];
  bool bad = false;
  float diag = 3.0e38f;
#pragma unroll
  for (int p = 0; p < QG; ++p) {
    float2 x = make_float2(0.f, 0.f);
    if (row && p < Q) {
      x = lane <= p ? G[size_t(lz_pidx(lane, p, Q)) * N + v]
                    : cconj(G[size_t(lz_pidx(p, lane, Q)) * N + v]);
      bad |= !isfinite(x.x) || !isfinite(x.y);
    }
    if (p == lane && row) {
      x.y = 0.f;
      diag = x.x;
    }
    g[p] = x;
  }
  if (bad && valid) atomicOr(status, PISCO_FLAG_NONFINITE);
  // start e_q*, q* = argmin_q G_qq (lowest q on ties)
  float best = diag;
  int bidx = row ? lane : QG;
#pragma unroll
  for (int off = QG / 2; off > 0; off >>= 1) {
    const float ob = __shfl_xor(best, off, QG);
    const int oi = __shfl_xor(bidx, off, QG);
    if (ob < best || (ob == best && oi < bidx)) {
      best = ob;
      bidx = oi;
    }
  }
  auto matvec = [&](float2 x) {
    float2 y = make_float2(0.f, 0.f);
#pragma unroll
    for (int p = 0; p < QG; ++p) {
      const float xr = __shfl(x.x, p, QG), xi = __shfl(x.y, p, QG);
      y.x = fmaf(g[p].x, xr, fmaf(-g[p].y, xi, y.x));
      y.y = fmaf(g[p].x, xi, fmaf(g[p].y, xr, y.y));
    }
    return y;
  };
  // w -= V (V^H w) over the first `cnt` basis vectors, twice
  auto reorth = [&](float2 w, int cnt) {
    for (int pass = 0; pass < 2; ++pass)
      for (int i = 0; i < cnt; ++i) {
        const float2 b = Vs[grp][i][lane];
        const float hr = lz_sum<QG>(b.x * w.x + b.y * w.y);
        const float hi = lz_sum<QG>(b.x * w.y - b.y * w.x);
        w.x -= hr * b.x - hi * b.y;
        w.y -= hr * b.y + hi * b.x;
      }
    return w;
  };
  // scale of the invariant-subspace test: bound, or (bound <= 0) the
  // voxel's largest row sum of |G| (at least its spectral radius)
  float scale = bound;
  if (!(bound > 0.f)) {
    float rs = 0.f;
#pragma unroll
    for (int p = 0; p < QG; ++p) rs += sqrtf(g[p].x * g[p].x + g[p].y * g[p].y);
#pragma unroll
    for (int off = QG / 2; off > 0; off >>= 1) rs = fmaxf(rs, __shfl_xor(rs, off, QG));
    scale = rs > 0.f ? rs : 1.f;
  }
  const float small = 1e-5f * scale;
  float2 x = make_float2(row && lane == bidx ? 1.f : 0.f, 0.f), prev = make_float2(0.f, 0.f);
  float beta = 0.f;
  for (int j = 0; j < K; ++j) {
    Vs[grp][j][lane] = x;
    float2 w = matvec(x);
    const float alpha = lz_sum<QG>(x.x * w.x + x.y * w.y);
    w.x -= alpha * x.x + beta * prev.x;
    w.y -= alpha * x.y + beta * prev.y;
    w = reorth(w, j + 1);
    float bn = sqrtf(lz_sum<QG>(w.x * w.x + w.y * w.y));
    if (lane == 0) {
      td[grp][j] = double(alpha);
      te[grp][j] = 0.0;
    }
    if (j + 1 == K) break;
    if (bn > small) {
      if (lane == 0) te[grp][j] = double(bn);
      prev = x;
      const float inv = 1.f / bn;
      x = make_float2(w.x * inv, w.y * inv);
      beta = bn;
    } else {
      // invariant subspace: continue from the next unit vector not in the
      // span of the basis (zero coupling in T)
      float2 y = make_float2(0.f, 0.f);
      float ny = 0.f;
      for (int t = 1; t <= Q && !(ny > 0.5f); ++t) {
        const int e = (bidx + j + t) % Q;
        y = reorth(make_float2(lane == e ? 1.f : 0.f, 0.f), j + 1);
        ny = sqrtf(lz_sum<QG>(y.x * y.x + y.y * y.y));
      }
      const float inv = ny > 0.f ? 1.f / ny : 0.f;
      x = make_float2(y.x * inv, y.y * inv);
      prev = make_float2(0.f, 0.f);
      beta = 0.f;
    }
  }
  // T's M smallest eigenpairs (FP64, the group's first lane), Ritz vectors
  float2 u[kMaxSets];
#pragma unroll
  for (int m = 0; m < kMaxSets; ++m) u[m] = make_float2(0.f, 0.f);
  double lo = 0.0, hi = 0.0, pivmin = DBL_MIN;
  if (lane == 0) {
    double emax2 = 0.0;
    for (int i = 0; i < K; ++i) {
      te2[grp][i] = te[grp][i] * te[grp][i];
      emax2 = fmax(emax2, te2[grp][i]);
    }
    pivmin = DBL_MIN * fmax(1.0, emax2);
    tri::gershgorin(td[grp], te[grp], K, &lo, &hi);
  }
#pragma unroll
  for (int m = 0; m < kMaxSets; ++m) {
    if (m >= M) break;
    if (lane == 0) {
      const double theta = tri::bisect(td[grp], te2[grp], K, m, lo, hi, pivmin, 0.0);
      th[grp][m] = theta;
      tri::twisted_vector(td[grp], te[grp], K, theta, pivmin, tw[grp][0], tw[grp][1], tz[grp]);
    }
    __syncthreads();
    float2 r = make_float2(0.f, 0.f);
    for (int i = 0; i < K; ++i) {
      const float zi = float(tz[grp][i]);
      const float2 b = Vs[grp][i][lane];
      r.x = fmaf(zi, b.x, r.x);
      r.y = fmaf(zi, b.y, r.y);
    }
    // orthogonal to the earlier sets (clusters of T), then unit norm
#pragma unroll
    for (int pass = 0; pass < 2; ++pass)
#pragma unroll
      for (int k = 0; k < kMaxSets; ++k) {
        if (k >= m) break;
        const float hr = lz_sum<QG>(u[k].x * r.x + u[k].y * r.y);
        const float hi2 = lz_sum<QG>(u[k].x * r.y - u[k].y * r.x);
        r.x -= hr * u[k].x - hi2 * u[k].y;
        r.y -= hr * u[k].y + hi2 * u[k].x;
      }
    const float nr = sqrtf(lz_sum<QG>(r.x * r.x + r.y * r.y));
    const float inv = nr > 0.f ? 1.f / nr : 0.f;
    r = make_float2(r.x * inv, r.y * inv);
    u[m] = r;
    __syncthreads();  // tz is rewritten for the next set
  }
  // Rayleigh quotients and residuals of the Ritz vectors
#pragma unroll
  for (int m = 0; m < kMaxSets; ++m) {
    if (m >= M) break;
    const float2 y = matvec(u[m]);
    const float l = lz_sum<QG>(u[m].x * y.x + u[m].y * y.y);
    const float rx = y.x - l * u[m].x, ry = y.y - l * u[m].y;
    const float rr = sqrtf(lz_sum<QG>(rx * rx + ry * ry));
    if (valid && row) maps[(size_t(m) * Q + lane) * N + v] = u[m];
    if (valid && lane == 0) {
      lam[size_t(m) * N + v] = l;
      if (resid) resid[size_t(m) * N + v] = rr;
    }
  }
}

}  // namespace

pisco_status_t run_eig_sets(Handle* h, int Q, long long N, float bound, int K, int M,
                            const float2* G, float2* maps, float* lam, float* resid) {
  if (N <= 0) return PISCO_OK;
#define PISCO_LANCZOS(QG)                                                                    \
  PISCO_KERNEL(h, k_lanczos<QG>, dim3(ceil_div(N, 256 / QG)), dim3(256), 0, G, Q, N, bound, \
               K, M, maps, lam, resid, h->status_dev)
  if (Q <= 4)
    PISCO_LANCZOS(4);
  else if (Q <= 8)
    PISCO_LANCZOS(8);
  else if (Q <= 16)
    PISCO_LANCZOS(16);
  else
    PISCO_LANCZOS(32);
#undef PISCO_LANCZOS
  return PISCO_OK;
}

}  // namespace pisco
