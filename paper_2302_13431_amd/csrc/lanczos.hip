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
// interval QG + 1 fold (QG / M + 1 fold for each of M sets).  Workgroups are dealt to
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

// a / b as a times the hardware reciprocal refined by one Newton step
// (relative error about 2e-15 from the estimate's 4.6e-8): four
// instructions in place of the ten of the IEEE division, in the Sturm counts
// and the twisted factorisation of T
struct FastDiv {
  __device__ static double div(double a, double b) {
    const double r0 = __builtin_amdgcn_rcp(b);
    const double e = fma(-b, r0, 1.0);
    return a * fma(r0, e, r0);
  }
};

// The twisted factorisation of tri::twisted_vector on two lanes: lane 0
// runs the top-down pivots D+ (kept in z) and multipliers Lp while lane 1
// runs the bottom-up pivots D- (kept in Dm) and multipliers Um; the twist
// r = argmin_i |gamma_i| (the largest such i, as the serial scan from the
// bottom takes it), gamma_i = D+_i + D-_i - (d_i - lambda), gamma_(n-1) =
// D+_(n-1); then lane 0 forms z above r and lane 1 below, and both scale
// their parts to unit norm.  Called by every lane of the group (the lanes
// past 1 only synchronise); z, Lp, Um, Dm are n-length LDS arrays.
__device__ inline void twisted2(const double* d, const double* e, int n, double lambda,
                                double pivmin, double* Lp, double* Um, double* Dm, double* z,
                                int lane) {
  if (n == 1) {
    if (lane == 0) z[0] = 1.0;
    wave_sync();
    return;
  }
  if (lane == 0) {
    double dp = d[0] - lambda;
    if (fabs(dp) < pivmin) dp = -pivmin;
    z[0] = dp;
    for (int i = 0; i + 1 < n; ++i) {
      Lp[i] = FastDiv::div(e[i], dp);
      dp = d[i + 1] - lambda - Lp[i] * e[i];
      if (fabs(dp) < pivmin) dp = -pivmin;
      z[i + 1] = dp;
    }
  } else if (lane == 1) {
    double dm = d[n - 1] - lambda;
    if (fabs(dm) < pivmin) dm = -pivmin;
    Dm[n - 1] = dm;
    for (int i = n - 1; i > 0; --i) {
      Um[i] = FastDiv::div(e[i - 1], dm);
      const double dn = d[i - 1] - lambda - Um[i] * e[i - 1];
      dm = fabs(dn) < pivmin ? -pivmin : dn;
      Dm[i - 1] = dm;
    }
  }
  wave_sync();
  int r = n - 1;
  if (lane < 2) {
    double best = fabs(z[n - 1]);
    for (int i = n - 2; i >= 0; --i) {
      const double gamma = z[i] + Dm[i] - (d[i] - lambda);
      if (fabs(gamma) < best) {
        best = fabs(gamma);
        r = i;
      }
    }
  }
  wave_sync();  // every lane has read the pivots before z is overwritten
  double s = 0.0;
  if (lane == 0) {
    double zi = 1.0;
    for (int i = r - 1; i >= 0; --i) {
      zi = -Lp[i] * zi;
      z[i] = zi;
      s += zi * zi;
    }
  } else if (lane == 1) {
    double zi = 1.0;
    for (int i = r + 1; i < n; ++i) {
      zi = -Um[i] * zi;
      z[i] = zi;
      s += zi * zi;
    }
  }
  if (lane < 2) Dm[lane] = s;  // partial sums of squares (Dm is free again)
  wave_sync();
  if (lane == 0) z[r] = 1.0;
  const double inv = 1.0 / sqrt(1.0 + Dm[0] + Dm[1]);
  wave_sync();
  if (lane == 0)
    for (int i = 0; i <= r; ++i) z[i] *= inv;
  else if (lane == 1)
    for (int i = r + 1; i < n; ++i) z[i] *= inv;
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
  __shared__ double th[NG][kMaxSets];
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
    constexpr int kIt = (NG * (QG * (QG + 1) / 2) + 63) / 64;  // loads per lane, at most
    float2* stage = &Vs[0][0][0];
    const int cnt = int((N - v0 < NG ? N - v0 : NG) * P);
    const float2* src = G + size_t(v0) * P;
    float2 tmp[kIt];
#pragma unroll
    for (int k = 0; k < kIt; ++k) {  // all loads in flight before the first store
      const int e = threadIdx.x + 64 * k;
      tmp[k] = e < cnt ? src[e] : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int k = 0; k < kIt; ++k) {
      const int e = threadIdx.x + 64 * k;
      if (e < NG * P) stage[e] = tmp[k];
    }
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
  // y = G x, x given by its QG components in LDS (16-byte aligned); four
  // partial sums keep four independent FMA chains in flight
  auto matvec = [&](const float2* xv) {
    const float4* x4 = reinterpret_cast<const float4*>(xv);
    float2 y[4] = {make_float2(0.f, 0.f), make_float2(0.f, 0.f), make_float2(0.f, 0.f),
                   make_float2(0.f, 0.f)};
#pragma unroll
    for (int p2 = 0; p2 < QG / 2; ++p2) {
      const float4 x = x4[p2];
      const float2 a = g[2 * p2], b = g[2 * p2 + 1];
      float2& u = y[(2 * p2) & 3];
      float2& w = y[(2 * p2 + 1) & 3];
      u.x = fmaf(a.x, x.x, fmaf(-a.y, x.y, u.x));
      u.y = fmaf(a.x, x.y, fmaf(a.y, x.x, u.y));
      w.x = fmaf(b.x, x.z, fmaf(-b.y, x.w, w.x));
      w.y = fmaf(b.x, x.w, fmaf(b.y, x.z, w.y));
    }
    return make_float2((y[0].x + y[1].x) + (y[2].x + y[3].x),
                       (y[0].y + y[1].y) + (y[2].y + y[3].y));
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
      float2 a[4] = {make_float2(0.f, 0.f), make_float2(0.f, 0.f), make_float2(0.f, 0.f),
                     make_float2(0.f, 0.f)};
#pragma unroll
      for (int p2 = 0; p2 < QG / 2; ++p2) {
        const float4 b = b4[p2], x = x4[p2];
        float2& u = a[(2 * p2) & 3];
        float2& t = a[(2 * p2 + 1) & 3];
        u.x = fmaf(b.x, x.x, fmaf(b.y, x.y, u.x));
        u.y = fmaf(b.x, x.y, fmaf(-b.y, x.x, u.y));
        t.x = fmaf(b.z, x.z, fmaf(b.w, x.w, t.x));
        t.y = fmaf(b.z, x.w, fmaf(-b.w, x.z, t.y));
      }
      h = make_float2((a[0].x + a[1].x) + (a[2].x + a[3].x),
                      (a[0].y + a[1].y) + (a[2].y + a[3].y));
    }
    wave_sync();
    xch[grp][lane] = h;  // zero beyond cnt
    wave_sync();
    float2 w1 = make_float2(0.f, 0.f);  // odd rows, summed apart
    for (int i0 = 0; i0 < cnt; i0 += CH) {
#pragma unroll
      for (int ii = 0; ii < CH; ii += 2) {
        const float4 hh = *reinterpret_cast<const float4*>(&xch[grp][i0 + ii]);
        const float2 b0 = Vs[grp][i0 + ii][lane], b1 = Vs[grp][i0 + ii + 1][lane];
        w.x -= hh.x * b0.x - hh.y * b0.y;
        w.y -= hh.x * b0.y + hh.y * b0.x;
        w1.x += hh.z * b1.x - hh.w * b1.y;
        w1.y += hh.z * b1.y + hh.w * b1.x;
      }
    }
    w.x -= w1.x;
    w.y -= w1.y;
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
  // T's M smallest eigenpairs in FP64.  The group's lanes share the
  // multisection of all M eigenvalues at once: set s takes lanes
  // [s W, s W + W), W = QG / M, one probe each per round (W + 1 fold), to an
  // absolute width of 1e-13 ||T|| (a twisted-factorisation vector is off by
  // about that width over the gap: 1e-8 at the closest pairs kept apart in
  // FP32, gaps of 1e-5 ||T||); lanes 0 and 1 then form each vector by the
  // twisted factorisation and all lanes form the Ritz vector.
  double emax2 = 0.0;
  for (int i = 0; i < K; ++i) {
    const double e = te[grp][i];
    emax2 = fmax(emax2, e * e);
  }
  if (lane < K) te2[grp][lane] = te[grp][lane] * te[grp][lane];
  const double pivmin = DBL_MIN * fmax(1.0, emax2);
  double glo, ghi;
  tri::gershgorin(td[grp], te[grp], K, &glo, &ghi);
  const double abstol = 1e-13 * fmax(fabs(glo), fabs(ghi));
  wave_sync();
  const unsigned long long gmask = ((1ull << QG) - 1ull) << (QG * grp);
  {
    const int W = QG / M, set = lane / W, k = lane - set * W;
    const bool mine = set < M;  // lanes past M W probe nothing of use
    const unsigned long long wmask = (1ull << W) - 1ull;
    double lo = glo, hi = ghi;
    for (int round = 0; round < 128; ++round) {
      const bool open = mine && hi - lo > abstol + 4.4e-16 * fmax(fabs(lo), fabs(hi));
      if (!(__ballot(open) & gmask)) break;
      const double step = (hi - lo) / double(W + 1);
      const int c = tri::negcount<FastDiv>(td[grp], te2[grp], K, lo + step * double(k + 1),
                                           pivmin);
      const unsigned long long above = (__ballot(mine && c > set) & gmask) >> (QG * grp);
      const unsigned long long seg = mine ? (above >> (set * W)) & wmask : 0ull;
      // first probe of the set above its eigenvalue (probe f at lo + (f + 1) step)
      double nlo, nhi;
      if (seg) {
        const int f = __ffsll((long long)seg) - 1;
        nhi = lo + step * double(f + 1);
        nlo = f > 0 ? lo + step * double(f) : lo;
      } else {
        nlo = lo + step * double(W);
        nhi = hi;
      }
      if (open) {
        if (nhi - nlo < hi - lo) {
          lo = nlo;
          hi = nhi;
        } else {  // no progress left in FP64
          lo = hi = 0.5 * (lo + hi);
        }
      }
    }
    if (mine && k == 0) th[grp][set] = 0.5 * (lo + hi);
  }
  wave_sync();
  float2 u[kMaxSets];
#pragma unroll
  for (int m = 0; m < kMaxSets; ++m) u[m] = make_float2(0.f, 0.f);
#pragma unroll
  for (int m = 0; m < kMaxSets; ++m) {
    if (m >= M) break;
    twisted2(td[grp], te[grp], K, th[grp][m], pivmin, tw[grp][0], tw[grp][1], te2[grp],
             tz[grp], lane);
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
