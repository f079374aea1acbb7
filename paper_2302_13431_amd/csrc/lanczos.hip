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
// from e_q* (q* = argmin_q G_qq), each the three-term recurrence followed by
// one classical Gram-Schmidt pass against the whole basis (full
// reorthogonalisation; the diagonal of T adds that pass's coefficient of the
// newest vector to alpha), the tridiagonal T = V^H G V eigen-decomposed in
// FP64 (multisection on Sturm counts, twisted factorisation), and the Ritz
// vectors of the M smallest Ritz values.  With K = Q the Krylov basis spans
// the whole space and the pairs are G's own to rounding.  A step whose new
// vector vanishes (an invariant subspace: G(x) has a large eigenspace at
// |Lambda|, so on real fields this happens in about half the steps; also the
// breakdown at the end of a smaller Krylov space) continues from the unit
// vector of the coordinate the basis covers least, orthogonalised against
// the basis, with a zero coupling in T.
//
// Mapping: a workgroup is one wave holding 64 / QG voxels, QG = next_pow2(Q)
// lanes each; lane q holds row q of G(x) in registers and component q of
// every vector.  G is read voxel-major, so that a workgroup's voxels are one
// contiguous block loaded by coalesced reads (the entry-major field of the
// G(x) stage is first copied so by a tiled transpose).  The Lanczos vectors live in LDS.  Cross-lane work goes
// through LDS instead of shuffles, in 16-byte reads where it can: a product
// reads the vector as broadcasts; a projection writes w, lane i forms
// <v_i, w> from row i, the coefficients are written back and every lane
// subtracts sum_i h_i v_i from its component.  One wave per workgroup lets
// the LDS exchanges be ordered without barriers.  The Sturm-count
// multisection spreads QG probes over the lanes, so every round narrows the
// interval QG + 1 fold.  Workgroups are dealt to
// the eight XCDs in contiguous voxel ranges, so that the lines of G(x) one
// workgroup reads are shared in its XCD's L2 with its neighbours.
#include <cfloat>

#include "common.hpp"
#include "tridiag.hpp"

namespace pisco {

namespace {

__device__ inline int lz_pidx(int p, int q, int Q) {  // p <= q
  return p * Q - p * (p - 1) / 2 + (q - p);
}

constexpr int kMaxSets = 8;
constexpr int kXcds = 8;

// Workgroup b of nb is dispatched to XCD b % 8; the logical index gives each
// XCD a contiguous range (a bijection on [0, nb)).
__device__ inline long long xcd_block(unsigned b, unsigned nb) {
  const unsigned x = b % kXcds, k = b / kXcds, q = nb / kXcds, r = nb % kXcds;
  const unsigned base = x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q;
  return (long long)base + k;
}

// G voxel-major: [N][Q(Q+1)/2], packed upper triangle of each voxel
template <int QG>
__global__ void __launch_bounds__(64) k_lanczos(const float2* __restrict__ G, int Q, long long N,
                                                float bound, int K, int M,
                                                float2* __restrict__ maps,
                                                float* __restrict__ lam,
                                                float* __restrict__ resid, unsigned* status) {
  constexpr int NG = 64 / QG;       // voxels per workgroup (one wave)
  constexpr int VS = QG + 2;        // padded row of the basis (16-byte aligned)
  constexpr int CH = QG < 8 ? QG : 8;  // rows per chunk of the projection update
  __shared__ __align__(16) float2 Vs[NG][QG][VS];  // [voxel][vector][component]
  __shared__ __align__(16) float2 xch[NG][QG];     // a vector or its coefficients
  __shared__ __align__(16) float red[NG][QG];
  __shared__ double td[NG][QG], te[NG][QG], te2[NG][QG], tz[NG][QG], tw[NG][2][QG];
  const int lane = threadIdx.x % QG, grp = threadIdx.x / QG;
  const long long v0 = xcd_block(blockIdx.x, gridDim.x) * NG;
  const long long vraw = v0 + grp;
  const bool valid = vraw < N;
  const long long v = valid ? vraw : N - 1;
  const bool row = lane < Q;
  const int P = Q * (Q + 1) / 2;
  // the workgroup's voxels are contiguous in the voxel-major input: staged
  // in the basis area by coalesced loads (zeros past N), then every lane
  // takes its row
  {
    float2* stage = &Vs[0][0][0];
    const int cnt = int((N - v0 < NG ? N - v0 : NG) * P);
    const float2* src = G + size_t(v0) * P;
    for (int e = threadIdx.x; e < NG * P; e += 64)
      stage[e] = e < cnt ? src[e] : make_float2(0.f, 0.f);
  }
  wave_sync();
  const float2* mine = &Vs[0][0][0] + grp * P;
  // row `lane` of G (zero beyond Q)
  float2 g[QG];
  bool bad = false;
  float diag = 3.0e38f;
#pragma unroll
  for (int p = 0; p < QG; ++p) {
    float2 x = make_float2(0.f, 0.f);
    if (row && p < Q) {
      x = lane <= p ? mine[lz_pidx(lane, p, Q)] : cconj(mine[lz_pidx(p, lane, Q)]);
      bad |= !isfinite(x.x) || !isfinite(x.y);
    }
    if (p == lane && row) {
      x.y = 0.f;
      diag = x.x;
    }
    g[p] = x;
  }
  if (bad && valid) atomicOr(status, PISCO_FLAG_NONFINITE);
  wave_sync();  // the staging area becomes the basis
  // rows not formed yet read as zeros (the projection update runs over
  // whole chunks of rows)
#pragma unroll
  for (int i = 0; i < QG; ++i) Vs[grp][i][lane] = make_float2(0.f, 0.f);

  // group sum of one value per lane, the same bits in every lane
  auto gsum = [&](float val) {
    red[grp][lane] = val;
    wave_sync();
    const float4* r4 = reinterpret_cast<const float4*>(red[grp]);
    float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
#pragma unroll
    for (int p = 0; p < QG / 4; ++p) {
      const float4 t = r4[p];
      s0 += t.x;
      s1 += t.y;
      s2 += t.z;
      s3 += t.w;
    }
    wave_sync();
    return (s0 + s1) + (s2 + s3);
  };
  // start e_q*, q* = argmin_q G_qq (lowest q on ties), from every lane's scan
  red[grp][lane] = diag;
  wave_sync();
  int bidx = 0;
  {
    float best = red[grp][0];
    for (int p = 1; p < Q; ++p) {
      const float d = red[grp][p];
      if (d < best) {
        best = d;
        bidx = p;
      }
    }
  }
  wave_sync();
  // y = G x, x given by its QG components in LDS (16-byte aligned)
  auto matvec = [&](const float2* xv) {
    const float4* x4 = reinterpret_cast<const float4*>(xv);
    float2 y = make_float2(0.f, 0.f);
#pragma unroll
    for (int p2 = 0; p2 < QG / 2; ++p2) {
      const float4 x = x4[p2];
      const float2 a = g[2 * p2], b = g[2 * p2 + 1];
      y.x = fmaf(a.x, x.x, fmaf(-a.y, x.y, y.x));
      y.y = fmaf(a.x, x.y, fmaf(a.y, x.x, y.y));
      y.x = fmaf(b.x, x.z, fmaf(-b.y, x.w, y.x));
      y.y = fmaf(b.x, x.w, fmaf(b.y, x.z, y.y));
    }
    return y;
  };
  // one classical Gram-Schmidt pass of w against rows 0..cnt-1 of Vs;
  // returns the new w and (in hl) the coefficient of row cnt - 1
  auto project = [&](float2 w, int cnt, float2* hl) {
    xch[grp][lane] = w;
    wave_sync();
    float2 h = make_float2(0.f, 0.f);
    if (lane < cnt) {
      const float4* b4 = reinterpret_cast<const float4*>(Vs[grp][lane]);
      const float4* x4 = reinterpret_cast<const float4*>(xch[grp]);
#pragma unroll
      for (int p2 = 0; p2 < QG / 2; ++p2) {
        const float4 b = b4[p2], x = x4[p2];
        h.x = fmaf(b.x, x.x, fmaf(b.y, x.y, h.x));
        h.y = fmaf(b.x, x.y, fmaf(-b.y, x.x, h.y));
        h.x = fmaf(b.z, x.z, fmaf(b.w, x.w, h.x));
        h.y = fmaf(b.z, x.w, fmaf(-b.w, x.z, h.y));
      }
    }
    wave_sync();
    xch[grp][lane] = h;  // zero beyond cnt
    wave_sync();
    for (int i0 = 0; i0 < cnt; i0 += CH) {
#pragma unroll
      for (int ii = 0; ii < CH; ii += 2) {
        const float4 hh = *reinterpret_cast<const float4*>(&xch[grp][i0 + ii]);
        const float2 b0 = Vs[grp][i0 + ii][lane], b1 = Vs[grp][i0 + ii + 1][lane];
        w.x -= hh.x * b0.x - hh.y * b0.y;
        w.y -= hh.x * b0.y + hh.y * b0.x;
        w.x -= hh.z * b1.x - hh.w * b1.y;
        w.y -= hh.z * b1.y + hh.w * b1.x;
      }
    }
    *hl = xch[grp][cnt - 1];
    wave_sync();
    return w;
  };
  // scale of the invariant-subspace test: bound, or (bound <= 0) the
  // voxel's largest row sum of |G| (at least its spectral radius)
  float scale = bound;
  if (!(bound > 0.f)) {
    float rs = 0.f;
#pragma unroll
    for (int p = 0; p < QG; ++p) rs += sqrtf(g[p].x * g[p].x + g[p].y * g[p].y);
    red[grp][lane] = rs;
    wave_sync();
    float mx = 0.f;
#pragma unroll
    for (int p = 0; p < QG; ++p) mx = fmaxf(mx, red[grp][p]);
    wave_sync();
    scale = mx > 0.f ? mx : 1.f;
  }
  const float small = 1e-5f * scale;
  // x: the newest basis vector, prev: the one before (zero after a restart);
  // cov: sum of |v_k[lane]|^2 over the basis so far (coverage of the lane's
  // coordinate)
  float2 x = make_float2(row && lane == bidx ? 1.f : 0.f, 0.f), prev = make_float2(0.f, 0.f);
  float beta = 0.f, cov = x.x;
  Vs[grp][0][lane] = x;
  for (int j = 0; j < K; ++j) {
    wave_sync();
    float2 w = matvec(Vs[grp][j]);
    // three-term recurrence, then one full reorthogonalisation pass
    const float alpha = gsum(x.x * w.x + x.y * w.y);
    w.x -= alpha * x.x + beta * prev.x;
    w.y -= alpha * x.y + beta * prev.y;
    float2 hj;
    w = project(w, j + 1, &hj);
    const float bn = sqrtf(gsum(w.x * w.x + w.y * w.y));
    const bool brk = !(bn > small);
    if (lane == 0) {
      td[grp][j] = double(alpha) + double(hj.x);
      te[grp][j] = (j + 1 < K && !brk) ? double(bn) : 0.0;
    }
    if (j + 1 == K) break;
    float2 xn = make_float2(0.f, 0.f);
    if (!brk) {
      const float inv = 1.f / bn;
      xn = make_float2(w.x * inv, w.y * inv);
    }
    // invariant subspace in some voxel: continue there from the unit vector
    // of the least covered coordinate e, orthogonalised against the basis
    // (zero coupling in T); it keeps ||(I - V V^H) e_e||^2 = 1 - cov_e >=
    // 1 - (j + 1) / Q of its norm.  Uniform over the wave; voxels that need
    // no vector ignore the result.
    if (__ballot(brk)) {
      red[grp][lane] = row ? cov : 3.0e38f;
      wave_sync();
      int e = 0;
      {
        float best = red[grp][0];
        for (int p = 1; p < Q; ++p) {
          const float c = red[grp][p];
          if (c < best) {
            best = c;
            e = p;
          }
        }
      }
      wave_sync();
      float2 y = make_float2(lane == e ? 1.f : 0.f, 0.f), hd;
      y = project(y, j + 1, &hd);
      y = project(y, j + 1, &hd);
      const float ny = sqrtf(gsum(y.x * y.x + y.y * y.y));
      if (brk && ny > 0.f) {
        const float inv = 1.f / ny;
        xn = make_float2(y.x * inv, y.y * inv);
      }
    }
    prev = brk ? make_float2(0.f, 0.f) : x;
    beta = brk ? 0.f : bn;
    x = xn;
    cov += x.x * x.x + x.y * x.y;
    Vs[grp][j + 1][lane] = x;
  }
  wave_sync();
  // T's M smallest eigenpairs in FP64: the group's lanes share the
  // multisection (one probe per lane and round), to an absolute width of
  // 4 eps ||T|| (the accuracy the twisted factorisation needs);
  // lane 0 forms the vector by the twisted factorisation; all lanes form the
  // Ritz vector
  double emax2 = 0.0;
  for (int i = 0; i < K; ++i) {
    const double e = te[grp][i];
    emax2 = fmax(emax2, e * e);
  }
  if (lane < K) te2[grp][lane] = te[grp][lane] * te[grp][lane];
  const double pivmin = DBL_MIN * fmax(1.0, emax2);
  double glo, ghi;
  tri::gershgorin(td[grp], te[grp], K, &glo, &ghi);
  const double abstol = 4.0 * DBL_EPSILON * fmax(fabs(glo), fabs(ghi));
  wave_sync();
  const unsigned long long gmask = ((1ull << QG) - 1ull) << (QG * grp);
  float2 u[kMaxSets];
#pragma unroll
  for (int m = 0; m < kMaxSets; ++m) u[m] = make_float2(0.f, 0.f);
#pragma unroll
  for (int m = 0; m < kMaxSets; ++m) {
    if (m >= M) break;
    double lo = glo, hi = ghi;
    for (int round = 0; round < 64; ++round) {
      if (hi - lo <= abstol + 4.4e-16 * fmax(fabs(lo), fabs(hi))) break;
      const double step = (hi - lo) / double(QG + 1);
      const int c = tri::negcount(td[grp], te2[grp], K, lo + step * double(lane + 1), pivmin);
      const unsigned long long above = (__ballot(c > m) & gmask) >> (QG * grp);
      // first probe above the m-th eigenvalue (probe f sits at lo + (f + 1) step)
      double nlo, nhi;
      if (above) {
        const int f = __ffsll((long long)above) - 1;
        nhi = lo + step * double(f + 1);
        nlo = f > 0 ? lo + step * double(f) : lo;
      } else {
        nlo = lo + step * double(QG);
        nhi = hi;
      }
      if (!(nhi - nlo < hi - lo)) break;  // no progress left in FP64
      lo = nlo;
      hi = nhi;
    }
    const double theta = 0.5 * (lo + hi);
    if (lane == 0)
      tri::twisted_vector(td[grp], te[grp], K, theta, pivmin, tw[grp][0], tw[grp][1], tz[grp]);
    wave_sync();
    float2 r = make_float2(0.f, 0.f);
    for (int i = 0; i < K; ++i) {
      const float zi = float(tz[grp][i]);
      const float2 b = Vs[grp][i][lane];
      r.x = fmaf(zi, b.x, r.x);
      r.y = fmaf(zi, b.y, r.y);
    }
    wave_sync();  // tz is rewritten for the next set
    // orthogonal to the earlier sets (clusters of T), then unit norm
#pragma unroll
    for (int pass = 0; pass < 2; ++pass)
#pragma unroll
      for (int k = 0; k < kMaxSets; ++k) {
        if (k >= m) break;
        const float hr = gsum(u[k].x * r.x + u[k].y * r.y);
        const float hi2 = gsum(u[k].x * r.y - u[k].y * r.x);
        r.x -= hr * u[k].x - hi2 * u[k].y;
        r.y -= hr * u[k].y + hi2 * u[k].x;
      }
    const float nr = sqrtf(gsum(r.x * r.x + r.y * r.y));
    const float inv = nr > 0.f ? 1.f / nr : 0.f;
    u[m] = make_float2(r.x * inv, r.y * inv);
  }
  // Rayleigh quotients and residuals of the Ritz vectors
#pragma unroll
  for (int m = 0; m < kMaxSets; ++m) {
    if (m >= M) break;
    xch[grp][lane] = u[m];
    wave_sync();
    const float2 y = matvec(xch[grp]);
    wave_sync();
    const float l = gsum(u[m].x * y.x + u[m].y * y.y);
    const float rx = y.x - l * u[m].x, ry = y.y - l * u[m].y;
    const float rr = sqrtf(gsum(rx * rx + ry * ry));
    if (valid && row) maps[(size_t(m) * Q + lane) * N + v] = u[m];
    if (valid && lane == 0) {
      lam[size_t(m) * N + v] = l;
      if (resid) resid[size_t(m) * N + v] = rr;
    }
  }
}

// Entry-major [P][N] -> voxel-major [N][P] through 32 x 64 LDS tiles: each
// row of a tile is read as 64 consecutive voxels of one entry (512 bytes),
// each voxel written as 32 consecutive entries (256 bytes).
__global__ void __launch_bounds__(256) k_voxel_major(const float2* __restrict__ G,
                                                     float2* __restrict__ Gt, int P,
                                                     long long N) {
  __shared__ float2 tile[32][65];
  const int t = threadIdx.x;
  const long long vb = blockIdx.x * 64LL;
  const int pb = blockIdx.y * 32;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int pr = t / 64 + 4 * k, vx = t % 64;
    if (pb + pr < P && vb + vx < N) tile[pr][vx] = G[size_t(pb + pr) * N + vb + vx];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int px = t % 32, vy = t / 32 + 8 * k;
    if (pb + px < P && vb + vy < N) Gt[size_t(vb + vy) * P + pb + px] = tile[px][vy];
  }
}

}  // namespace

size_t layout_eig_sets(int Q, long long N) {
  return size_t(Q) * (Q + 1) / 2 * size_t(N) * sizeof(float2) + 256;
}

pisco_status_t run_lanczos_vm(Handle* h, int Q, long long N, float bound, int K, int M,
                              const float2* Gvm, float2* maps, float* lam, float* resid) {
  if (N <= 0) return PISCO_OK;
#define PISCO_LANCZOS(QG)                                                                   \
  PISCO_KERNEL(h, k_lanczos<QG>, dim3(ceil_div(N, 64 / QG)), dim3(64), 0, Gvm, Q, N, bound, \
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

pisco_status_t run_eig_sets(Handle* h, int Q, long long N, float bound, int K, int M,
                            const float2* G, float2* maps, float* lam, float* resid, void* ws) {
  if (N <= 0) return PISCO_OK;
  const int P = Q * (Q + 1) / 2;
  float2* Gvm = static_cast<float2*>(ws);
  PISCO_KERNEL(h, k_voxel_major, dim3(ceil_div(N, 64), ceil_div(P, 32)), dim3(256), 0, G, Gvm,
               P, N);
  return run_lanczos_vm(h, Q, N, bound, K, M, Gvm, maps, lam, resid);
}

}  // namespace pisco
