// Eigen-decomposition of the small Hermitian Rayleigh-Ritz matrix H = X^H A X
// (order b, FP64) used by the signal/null split.
//
//   k_hetrd_reg / k_hetrd_step: Householder reduction H = Q T Q^H with T
//                 real symmetric tridiagonal (each reflector H_k = I - tau_k
//                 v_k v_k^H is chosen so that H_k^H maps the column below the
//                 diagonal onto a real multiple of the first unit vector); the
//                 reflectors are kept for the back-transformation.  Up to
//                 order 128 one workgroup holds the matrix in registers
//                 (k_hetrd_reg); beyond that one launch per step spreads the
//                 matrix's columns over many workgroups (k_hetrd_step).
//   k_tri_eigval  one workgroup per eigenvalue: multisection on Sturm counts
//                 (256 points per step), to about eps * ||T||.
//   k_tri_vector  one workgroup per eigenvalue: the eigenvector of T by the
//                 twisted factorisation; eigenvalues closer than 1e-12 ||T||
//                 (and the rare vector whose residual is not small) go to
//                 inverse iteration with Gram-Schmidt inside the cluster.  The
//                 vector is then mapped back, u = Q z, by one wave holding its
//                 rows in registers, and written in descending eigenvalue
//                 order.
//
// Cost for b = 96: b - 1 reduction steps of four barriers each, then
// independent per-eigenvalue work spread over b workgroups.  The former
// one-sided Jacobi needed about seven sweeps of b - 1 barrier rounds for the
// Rayleigh-Ritz matrices met here (far from diagonal).
#include <cfloat>

#include "common.hpp"
#include "tridiag.hpp"

namespace pisco {

namespace {

constexpr int kTrdLdsMax = 96;   // largest b reduced with twelve register columns per thread
constexpr int kTriMax = 1024;    // largest b of the tridiagonal kernels

// Sum over the 64 lanes of a wave (all lanes active), every lane getting
// the total: an inclusive scan within each row of 16 lanes by DPP moves
// (row_shr 1, 2, 4, 8), then row_bcast:15 into rows 1 and 3 and
// row_bcast:31 into rows 2 and 3, so that lane 63 holds the sum, read back
// with readlane.  No LDS round trips.
template <int kCtrl, int kRowMask>
__device__ inline double dpp_f64(double v) {
  const long long x = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, int(x), kCtrl, kRowMask, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, int(x >> 32), kCtrl, kRowMask, 0xf, true);
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned>(lo));
}
__device__ inline double wave_sum(double v) {
  v += dpp_f64<0x111, 0xf>(v);  // row_shr:1
  v += dpp_f64<0x112, 0xf>(v);  // row_shr:2
  v += dpp_f64<0x114, 0xf>(v);  // row_shr:4
  v += dpp_f64<0x118, 0xf>(v);  // row_shr:8
  v += dpp_f64<0x142, 0xa>(v);  // row_bcast:15
  v += dpp_f64<0x143, 0xc>(v);  // row_bcast:31
  const long long x = __double_as_longlong(v);
  const unsigned lo = __builtin_amdgcn_readlane(int(x), 63);
  const unsigned hi = __builtin_amdgcn_readlane(int(x >> 32), 63);
  return __longlong_as_double((static_cast<long long>(hi) << 32) | lo);
}
__device__ inline double wave_max(double v) {
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}
__device__ inline double wave_min(double v) {
  for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
  return v;
}

// ------------------------------------------------------------------ reduction

// A = (H + H^H) / 2, column-major (the stepped reduction's first buffer).
__global__ void k_hetrd_sym(const double2* __restrict__ H, int b, double2* __restrict__ A) {
  const long long e = blockIdx.x * 256LL + threadIdx.x;
  if (e >= 1LL * b * b) return;
  const int i = int(e % b), j = int(e / b);
  const double2 x = H[e], y = H[size_t(i) * b + j];
  A[e] = make_double2(0.5 * (x.x + y.x), 0.5 * (x.y - y.y));
}

// Step k of the reduction for orders above 128 (one launch per step, k = 0
// .. b - 1), on one-wave workgroups that each own every gridDim.x-th column
// of the trailing block.  With A^(k) the matrix after k reflections and
// x_{k-1} = tau_{k-1} A^(k-1)_22 v_{k-1} from the previous launch, every
// workgroup forms the same w_{k-1} = x - (tau/2)(x^H v) v, the updated column
// k of A^(k) and from it the reflector (v_k, tau_k, beta_k) (workgroup 0
// stores them, with d_k and e_k = beta_k); then each applies
// A^(k) = A^(k-1) - v w^H - w v^H to its own columns (rows > k), writes them
// to the other buffer and forms x_k for them: by Hermitian symmetry
// (A v)_j = sum_i conj(A_ij) v_i, a dot product down its own column, so no
// sum crosses workgroups.  x_{k-1} and x_k sit in two vectors (every
// workgroup reads the one while some write the other); b <= 64 kR.
template <int kR>
__global__ void __launch_bounds__(64) k_hetrd_step(const double2* __restrict__ Aold,
                                                   double2* __restrict__ Anew, int b, int k,
                                                   const double2* __restrict__ xin,
                                                   double2* __restrict__ xout,
                                                   double2* __restrict__ refl,
                                                   double2* __restrict__ tau_out,
                                                   double* __restrict__ d_out,
                                                   double* __restrict__ e_out) {
  constexpr int kMaxB = 64 * kR;
  __shared__ double2 vpS[kMaxB], wpS[kMaxB], vS[kMaxB], cS[kMaxB];
  const int lane = threadIdx.x;
  // previous reflector and its w on rows k .. b - 1
  if (k >= 1) {
    const int kp = k - 1;
    const double2 tp = tau_out[kp];
    double2 xr[kR], vr[kR];
    double dr = 0.0, di = 0.0;
#pragma unroll
    for (int s = 0; s < kR; ++s) {
      const int i = k + lane + 64 * s;
      xr[s] = make_double2(0.0, 0.0);
      vr[s] = make_double2(0.0, 0.0);
      if (i < b) {
        vr[s] = refl[size_t(kp) * b + i];
        xr[s] = xin[i];
        dr += xr[s].x * vr[s].x + xr[s].y * vr[s].y;
        di += xr[s].x * vr[s].y - xr[s].y * vr[s].x;
      }
    }
    dr = wave_sum(dr);
    di = wave_sum(di);
    const double2 ap = zmul(make_double2(-0.5 * tp.x, -0.5 * tp.y), make_double2(dr, di));
#pragma unroll
    for (int s = 0; s < kR; ++s) {
      const int i = k + lane + 64 * s;
      if (i < b) {
        vpS[i] = vr[s];
        wpS[i] = zadd(xr[s], zmul(ap, vr[s]));
      }
    }
  }
  __syncthreads();
  // column k of A^(k) on rows k .. b - 1
  const double2 vk = k >= 1 ? vpS[k] : make_double2(0.0, 0.0);
  const double2 wk = k >= 1 ? wpS[k] : make_double2(0.0, 0.0);
#pragma unroll
  for (int s = 0; s < kR; ++s) {
    const int i = k + lane + 64 * s;
    if (i < b) {
      double2 a = Aold[size_t(k) * b + i];
      if (k >= 1) {
        const double2 vi = vpS[i], wi = wpS[i];
        a.x -= vi.x * wk.x + vi.y * wk.y + wi.x * vk.x + wi.y * vk.y;
        a.y -= vi.y * wk.x - vi.x * wk.y + wi.y * vk.x - wi.x * vk.y;
      }
      cS[i] = a;
    }
  }
  __syncthreads();
  const bool lead = blockIdx.x == 0;
  if (k + 1 >= b) {  // the last diagonal entry only
    if (lead && lane == 0) {
      d_out[k] = cS[k].x;
      e_out[k] = 0.0;
    }
    return;
  }
  // reflector from rows k + 1 .. b - 1 (the arithmetic of k_hetrd_reg)
  double sq = 0.0;
#pragma unroll
  for (int s = 0; s < kR; ++s) {
    const int i = k + 2 + lane + 64 * s;
    if (i < b) sq += zabs2(cS[i]);
  }
  sq = wave_sum(sq);
  const double2 al = cS[k + 1];
  double2 tau = make_double2(0.0, 0.0), scale = make_double2(0.0, 0.0);
  double beta = al.x;
  if (sq > 0.0 || al.y != 0.0) {
    const double nrm = sqrt(zabs2(al) + sq);
    beta = al.x >= 0.0 ? -nrm : nrm;
    tau = make_double2((beta - al.x) / beta, -al.y / beta);
    const double2 den = make_double2(al.x - beta, al.y);  // |den| >= nrm
    const double inv = 1.0 / zabs2(den);
    scale = make_double2(den.x * inv, -den.y * inv);
  }
#pragma unroll
  for (int s = 0; s < kR; ++s) {
    const int i = k + 1 + lane + 64 * s;
    if (i < b) {
      const double2 v = i == k + 1 ? make_double2(1.0, 0.0) : zmul(cS[i], scale);
      vS[i] = v;
      if (lead) refl[size_t(k) * b + i] = v;
    }
  }
  if (lead && lane == 0) {
    tau_out[k] = tau;
    e_out[k] = beta;
    d_out[k] = cS[k].x;
  }
  __syncthreads();
  // own columns: update (rows > k), store, and x_k = tau A^(k) v_k there
  for (int j = k + 1 + blockIdx.x; j < b; j += gridDim.x) {
    const double2 vj = k >= 1 ? vpS[j] : make_double2(0.0, 0.0);
    const double2 wj = k >= 1 ? wpS[j] : make_double2(0.0, 0.0);
    double pr = 0.0, pi = 0.0;
#pragma unroll
    for (int s = 0; s < kR; ++s) {
      const int i = k + 1 + lane + 64 * s;
      if (i < b) {
        double2 a = Aold[size_t(j) * b + i];
        if (k >= 1) {
          const double2 vi = vpS[i], wi = wpS[i];
          a.x -= vi.x * wj.x + vi.y * wj.y + wi.x * vj.x + wi.y * vj.y;
          a.y -= vi.y * wj.x - vi.x * wj.y + wi.y * vj.x - wi.x * vj.y;
          Anew[size_t(j) * b + i] = a;
        }
        const double2 v = vS[i];
        pr += a.x * v.x + a.y * v.y;  // conj(a) v
        pi += a.x * v.y - a.y * v.x;
      }
    }
    pr = wave_sum(pr);
    pi = wave_sum(pi);
    if (lane == 0) xout[j] = zmul(tau, make_double2(pr, pi));
  }
}


// The reduction for b <= 8 kU with A held in registers: thread t owns
// row i = t % 128 of the columns j = sl + 8 u (sl = t / 128, u < kU; kU = 12
// for b <= 96, 16 for b <= 128).
// The product and the rank-2 update then read only v and w (broadcast) from
// LDS, and the column the next reflector is built from is passed through
// LDS by its owners.  v and w are zero outside rows k+1 .. b-1, so the
// update leaves the eliminated rows and columns alone without a branch;
// groups of four columns that are all eliminated are skipped (uniform per
// wave).
template <int kU>
__global__ void __launch_bounds__(1024) k_hetrd_reg(const double2* __restrict__ H, int b,
                                                    double2* __restrict__ refl,
                                                    double2* __restrict__ tau_out,
                                                    double* __restrict__ d_out,
                                                    double* __restrict__ e_out) {
  // column groups of four, or two where sixteen columns leave fewer registers
  constexpr int kR = 128, kS = 8, kN = kS * kU, kG = kU > 12 ? 2 : 4;
  static_assert(kU % kG == 0 && kN <= kR, "column groups");
  __shared__ double2 colbuf[kN];
  __shared__ double2 part[kS][kN];
  __shared__ double2 vs[kN], ws[kN];
  __shared__ double2 sh_tau;
  const int t = threadIdx.x, i = t % kR, sl = t / kR;
  const bool rowok = i < b;
  const double2 zero = make_double2(0.0, 0.0);
  double2 a[kU];
#pragma unroll
  for (int u = 0; u < kU; ++u) {
    const int j = sl + kS * u;
    a[u] = zero;
    if (rowok && j < b) {
      const double2 x = H[size_t(j) * b + i], y = H[size_t(i) * b + j];
      a[u] = make_double2(0.5 * (x.x + y.x), 0.5 * (x.y - y.y));
    }
  }
  if (t < kN) {
    vs[t] = zero;
    ws[t] = zero;
  }
  if (sl == 0 && rowok) colbuf[i] = a[0];
  __syncthreads();
  for (int k = 0; k + 1 < b; ++k) {
    if (t < 64) {
      double s = 0.0;
      for (int r = k + 2 + t; r < b; r += 64) s += zabs2(colbuf[r]);
      s = wave_sum(s);
      const double2 al = colbuf[k + 1];
      double2 tau = zero, scale = zero;
      double beta = al.x;
      if (s > 0.0 || al.y != 0.0) {
        const double nrm = sqrt(zabs2(al) + s);
        beta = al.x >= 0.0 ? -nrm : nrm;
        tau = make_double2((beta - al.x) / beta, -al.y / beta);
        const double2 den = make_double2(al.x - beta, al.y);  // |den| >= nrm
        const double inv = 1.0 / zabs2(den);
        scale = make_double2(den.x * inv, -den.y * inv);
      }
      for (int r = t; r < b; r += 64) {
        const double2 v = r <= k ? zero : r == k + 1 ? make_double2(1.0, 0.0)
                                                     : zmul(colbuf[r], scale);
        vs[r] = v;
        if (r > k) refl[size_t(k) * b + r] = v;
      }
      if (t == 0) {
        sh_tau = tau;
        tau_out[k] = tau;
        e_out[k] = beta;
        d_out[k] = colbuf[k].x;
      }
    }
    __syncthreads();
    const double2 tau = sh_tau;
    {
      double2 acc = zero;
#pragma unroll
      for (int g = 0; g < kU / kG; ++g) {
        if (sl + kS * (kG * g + kG - 1) > k) {
          double2 v[kG];
#pragma unroll
          for (int uu = 0; uu < kG; ++uu) v[uu] = vs[sl + kS * (kG * g + uu)];
#pragma unroll
          for (int uu = 0; uu < kG; ++uu) {
            const double2 x = a[kG * g + uu];
            acc.x += x.x * v[uu].x - x.y * v[uu].y;
            acc.y += x.x * v[uu].y + x.y * v[uu].x;
          }
        }
      }
      if (rowok) part[sl][i] = acc;
    }
    __syncthreads();
    if (t < 64) {
      double dr = 0.0, di = 0.0;  // x^H v
      for (int r = t; r < b; r += 64) {
        double2 x = part[0][r];
#pragma unroll
        for (int q = 1; q < kS; ++q) x = zadd(x, part[q][r]);
        x = zmul(tau, x);
        part[0][r] = x;
        const double2 v = vs[r];
        dr += x.x * v.x + x.y * v.y;
        di += x.x * v.y - x.y * v.x;
      }
      dr = wave_sum(dr);
      di = wave_sum(di);
      const double2 ap = zmul(make_double2(-0.5 * tau.x, -0.5 * tau.y), make_double2(dr, di));
      for (int r = t; r < b; r += 64)
        ws[r] = r <= k ? zero : zadd(part[0][r], zmul(ap, vs[r]));
    }
    __syncthreads();
    {
      const double2 vi = rowok ? vs[i] : zero, wi = rowok ? ws[i] : zero;
#pragma unroll
      for (int g = 0; g < kU / kG; ++g) {
        if (sl + kS * (kG * g + kG - 1) > k) {
          double2 vj[kG], wj[kG];
#pragma unroll
          for (int uu = 0; uu < kG; ++uu) {
            vj[uu] = vs[sl + kS * (kG * g + uu)];
            wj[uu] = ws[sl + kS * (kG * g + uu)];
          }
#pragma unroll
          for (int uu = 0; uu < kG; ++uu) {
            double2& x = a[kG * g + uu];
            x.x -= vi.x * wj[uu].x + vi.y * wj[uu].y + wi.x * vj[uu].x + wi.y * vj[uu].y;
            x.y -= vi.y * wj[uu].x - vi.x * wj[uu].y + wi.y * vj[uu].x - wi.x * vj[uu].y;
          }
        }
      }
      // column k + 1 to LDS for the next reflector
      const int jn = k + 1;
      if (rowok && sl == jn % kS) {
        const int un = jn / kS;
#pragma unroll
        for (int u = 0; u < kU; ++u)
          if (u == un) colbuf[i] = a[u];
      }
    }
    __syncthreads();
  }
  if (t == 0) {
    d_out[b - 1] = colbuf[b - 1].x;
    e_out[b - 1] = 0.0;
  }
}

// ------------------------------------------------------------------ eigenvalues

// Eigenvalue j (ascending, 0-based) of T by multisection: each of the
// kEigThreads lanes of the workgroup takes the Sturm count at one of
// kEigThreads interior points of the bracket (8 bits per step with 256).
// The waves' ballots meet in LDS (double-buffered: one barrier per step);
// every lane recomputes the chosen points from their formula.
// The Sturm count of tri::negcount (the same arithmetic in the same order,
// so the same count), with eight steps' operands read from LDS at once, so
// that the chain of divisions waits on LDS once per chunk.
__device__ inline int negcount_chunked(const double* d, const double* e2, int n, double x,
                                       double pivmin) {
  int c = 0;
  double q = d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  c += q < 0.0;
  constexpr int kChunk = 8;
  auto step = [&](double di, double ei) {
    q = di - x - ei / q;
    if (fabs(q) < pivmin) q = -pivmin;
    c += q < 0.0;
  };
  int i = 1;
  for (; i + kChunk <= n; i += kChunk) {
    double dc[kChunk], ec[kChunk];
#pragma unroll
    for (int u = 0; u < kChunk; ++u) {
      dc[u] = d[i + u];
      ec[u] = e2[i + u - 1];
    }
#pragma unroll
    for (int u = 0; u < kChunk; ++u) step(dc[u], ec[u]);
  }
  for (; i < n; ++i) step(d[i], e2[i - 1]);
  return c;
}

constexpr int kEigThreads = 256;
__global__ void __launch_bounds__(kEigThreads) k_tri_eigval(const double* __restrict__ d,
                                                            const double* __restrict__ e,
                                                            int b, double* __restrict__ lam) {
  constexpr int kW = kEigThreads / 64;
  __shared__ double sd[kTriMax], se2[kTriMax];
  __shared__ double red[3][kW];
  __shared__ unsigned long long masks[2][kW];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6, j = blockIdx.x;
  double glo = INFINITY, ghi = -INFINITY, emax2 = 0.0;
  for (int i = t; i < b; i += kEigThreads) {
    const double di = d[i];
    const double el = i > 0 ? e[i - 1] : 0.0, er = i + 1 < b ? e[i] : 0.0;
    sd[i] = di;
    se2[i] = er * er;
    emax2 = fmax(emax2, er * er);
    const double r = fabs(el) + fabs(er);
    glo = fmin(glo, di - r);
    ghi = fmax(ghi, di + r);
  }
  glo = wave_min(glo);
  ghi = wave_max(ghi);
  emax2 = wave_max(emax2);
  if (lane == 0) {
    red[0][wave] = glo;
    red[1][wave] = ghi;
    red[2][wave] = emax2;
  }
  __syncthreads();
#pragma unroll
  for (int w = 0; w < kW; ++w) {
    glo = fmin(glo, red[0][w]);
    ghi = fmax(ghi, red[1][w]);
    emax2 = fmax(emax2, red[2][w]);
  }
  const double pivmin = DBL_MIN * fmax(1.0, emax2);
  const double wide = 2.0 * DBL_EPSILON * fmax(fabs(glo), fabs(ghi)) + 2.0 * pivmin;
  double lo = glo - wide, hi = ghi + wide;
  constexpr double kInv = 1.0 / double(kEigThreads + 1);
  for (int it = 0; it < 64; ++it) {
    const double w = hi - lo;
    if (!(w > 2.0 * DBL_EPSILON * fmax(fabs(lo), fabs(hi)) + 4.0 * pivmin)) break;
    auto point = [&](int q) { return lo + w * (double(q + 1) * kInv); };
    const int c = negcount_chunked(sd, se2, b, point(t), pivmin);
    const unsigned long long mk = __ballot(c > j);
    if (lane == 0) masks[it & 1][wave] = mk;
    __syncthreads();
    int l = kEigThreads;  // first point whose count exceeds j
#pragma unroll
    for (int q = kW - 1; q >= 0; --q) {
      const unsigned long long m = masks[it & 1][q];
      if (m) l = 64 * q + __builtin_ctzll(m);
    }
    const double nlo = l == 0 ? lo : point(l - 1);
    const double nhi = l == kEigThreads ? hi : point(l);
    if (nlo == lo && nhi == hi) break;
    lo = nlo;
    hi = nhi;
  }
  if (t == 0) lam[j] = 0.5 * (lo + hi);
}

// ------------------------------------------------------------------ eigenvectors

// z <- z / ||z||_2 over the b entries in LDS (wave 0 only), scaled by the
// largest magnitude first so that no square overflows.
__device__ void wave_normalize(double* z, int b) {
  const int t = threadIdx.x;
  double mx = 0.0;
  for (int i = t; i < b; i += 64) mx = fmax(mx, fabs(z[i]));
  mx = wave_max(mx);
  const double s1 = mx > 0.0 ? 1.0 / mx : 1.0;
  double ss = 0.0;
  for (int i = t; i < b; i += 64) {
    const double v = z[i] * s1;
    ss += v * v;
  }
  ss = wave_sum(ss);
  const double s2 = ss > 0.0 ? s1 / sqrt(ss) : 0.0;
  for (int i = t; i < b; i += 64) z[i] *= s2;
  __syncthreads();
}

// u = Q z for the real tridiagonal eigenvector z (LDS), written as column
// `col` of U (b x b column-major).  Lane t keeps rows t + 64 q in registers;
// the reflectors are applied last to first.
template <int kPL>
__device__ __attribute__((always_inline)) void back_transform(const double* z, int b,
                                                              const double2* __restrict__ refl,
                                                              const double2* __restrict__ tau,
                                                              double2* __restrict__ U, int col) {
  // reflectors come from global memory kDepth - 1 steps ahead of their use
  // (a ring of registers, each slot refilled right after its step), so that
  // the chain of steps does not wait on the L2
  constexpr int kDepth = kPL <= 2 ? 8 : 1;
  const int t = threadIdx.x;
  double2 u[kPL];
#pragma unroll
  for (int q = 0; q < kPL; ++q) {
    const int r = t + 64 * q;
    u[q] = make_double2(r < b ? z[r] : 0.0, 0.0);
  }
  // loads are unconditional (a clamped, valid address) and the entries
  // outside the reflector are zeroed where they are used: a predicated load
  // would make every later use wait for all the loads in flight
  auto load = [&](int k, double2 (&vq)[kPL], double2& tk) {
    const int kc = k >= 0 ? k : 0;
    tk = tau[kc];
    const double2* v = refl + size_t(kc) * b;
#pragma unroll
    for (int q = 0; q < kPL; ++q) {
      const int r = t + 64 * q;
      vq[q] = v[r < b ? r : b - 1];
    }
  };
  // one reflector step; a zero tau gives ts = 0 and leaves u unchanged, so
  // the step has no branch (a branch would make the loop wait for every load
  // in flight where its paths join)
  auto apply = [&](int k, const double2 (&ring_k)[kPL], double2 tk) {
    double2 vq[kPL];
#pragma unroll
    for (int q = 0; q < kPL; ++q) {
      const int r = t + 64 * q;
      const bool in = r > k && r < b;  // the reflector's rows
      vq[q] = make_double2(in ? ring_k[q].x : 0.0, in ? ring_k[q].y : 0.0);
    }
    double sr = 0.0, si = 0.0;  // v^H u
#pragma unroll
    for (int q = 0; q < kPL; ++q) {
      sr += vq[q].x * u[q].x + vq[q].y * u[q].y;
      si += vq[q].x * u[q].y - vq[q].y * u[q].x;
    }
    sr = wave_sum(sr);
    si = wave_sum(si);
    const double2 ts = zmul(tk, make_double2(sr, si));
#pragma unroll
    for (int q = 0; q < kPL; ++q) u[q] = zsub(u[q], zmul(vq[q], ts));
  };
  double2 ring[kDepth][kPL], tr[kDepth];
#pragma unroll
  for (int dd = 0; dd < kDepth; ++dd) load(b - 2 - dd, ring[dd], tr[dd]);
  // whole groups of kDepth steps (k = b-2 down to b-1-ngrp*kDepth), then the
  // remaining steps down to k = 0
  const int ngrp = (b - 1) / kDepth;
  int k0 = b - 2;
  for (int g = 0; g < ngrp; ++g, k0 -= kDepth) {
#pragma unroll
    for (int dd = 0; dd < kDepth; ++dd) {
      const int k = k0 - dd;
      apply(k, ring[dd], tr[dd]);
      load(k - kDepth, ring[dd], tr[dd]);
    }
  }
#pragma unroll
  for (int dd = 0; dd < kDepth; ++dd)
    if (k0 - dd >= 0) apply(k0 - dd, ring[dd], tr[dd]);
#pragma unroll
  for (int q = 0; q < kPL; ++q) {
    const int r = t + 64 * q;
    if (r < b) U[size_t(col) * b + r] = u[q];
  }
}

// Eigenvector z of T for lambda by the twisted factorisation, the same
// arithmetic as tri::twisted_vector but on one wave: the top-down pivots
// D+ and ratios L+ (lane 0) and the bottom-up D- and U- (lane 1) run side by
// side, the twist index (smallest |gamma|, the larger index on ties) is a
// wave reduction, the two outward recurrences for z again run on lanes 0
// and 1, and the norm is a wave sum.  Lp, Um, Dp, Dm are n-length LDS
// scratch, distinct from d, e and z (restrict: the next step's loads need
// not wait behind this step's stores); all 64 lanes call it.
__device__ void twisted_vector_wave(const double* __restrict__ d, const double* __restrict__ e,
                                    int n, double lambda, double pivmin, double* __restrict__ Lp,
                                    double* __restrict__ Um, double* __restrict__ Dp,
                                    double* __restrict__ Dm, double* __restrict__ z) {
  const int t = threadIdx.x;
  if (n == 1) {
    if (t == 0) z[0] = 1.0;
    __syncthreads();
    return;
  }
  if (t < 2) {
    const bool up = t == 1;
    double q = d[up ? n - 1 : 0] - lambda;
    if (fabs(q) < pivmin) q = -pivmin;
    (up ? Dm : Dp)[up ? n - 1 : 0] = q;
    // step s uses the off-diagonal entry ie(s) and the diagonal entry id(s)
    // of the new pivot; the pairs of kChunk steps are read together, so that
    // the chain of divisions waits on LDS once per chunk, and the stores go
    // through a selected address, so that the steps have no branch
    auto ie = [&](int st) { return up ? n - 2 - st : st; };
    auto id = [&](int st) { return up ? n - 2 - st : st + 1; };
    auto step = [&](int st, double ec, double dc) {
      const double ratio = ec / q;
      double nq = dc - lambda - ratio * ec;
      if (fabs(nq) < pivmin) nq = -pivmin;
      double* rp = up ? Um + (n - 1 - st) : Lp + st;
      double* pp = up ? Dm + id(st) : Dp + id(st);
      *rp = ratio;
      *pp = nq;
      q = nq;
    };
    constexpr int kChunk = 8;
    int st = 0;
    for (; st + kChunk <= n - 1; st += kChunk) {
      double ec[kChunk], dc[kChunk];
#pragma unroll
      for (int u = 0; u < kChunk; ++u) {
        ec[u] = e[ie(st + u)];
        dc[u] = d[id(st + u)];
      }
#pragma unroll
      for (int u = 0; u < kChunk; ++u) step(st + u, ec[u], dc[u]);
    }
    for (; st + 1 < n; ++st) step(st, e[ie(st)], d[id(st)]);
  }
  __syncthreads();
  // twist: gamma_{n-1} = D+(n-1), gamma_i = D+(i) + D-(i) - (d_i - lambda)
  double best = INFINITY;
  int r = -1;
  for (int i = t; i < n; i += 64) {
    const double g = i == n - 1 ? fabs(Dp[n - 1]) : fabs(Dp[i] + Dm[i] - (d[i] - lambda));
    if (g < best || (g == best && i > r)) {
      best = g;
      r = i;
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    const double ob = __shfl_xor(best, off, 64);
    const int orr = __shfl_xor(r, off, 64);
    if (ob < best || (ob == best && orr > r)) {
      best = ob;
      r = orr;
    }
  }
  if (r < 0) r = n - 1;  // every gamma NaN: the sequential rule keeps n - 1
  for (int i = t; i < n; i += 64) z[i] = i == r ? 1.0 : 0.0;
  __syncthreads();
  if (t < 2) {
    const bool up = t == 1;
    const int len = up ? n - 1 - r : r;
    double zz = 1.0;
    for (int s = 0; s < len; ++s) {
      const int i = up ? r + 1 + s : r - 1 - s;
      zz = -(up ? Um[i] : Lp[i]) * zz;
      z[i] = zz;
    }
  }
  __syncthreads();
  double ss = 0.0;
  for (int i = t; i < n; i += 64) ss += z[i] * z[i];
  ss = wave_sum(ss);
  const double inv = 1.0 / sqrt(ss);
  for (int i = t; i < n; i += 64) z[i] *= inv;
  __syncthreads();
}

// One workgroup (one wave) per eigenvalue j.  Members of a cluster (gaps
// below 1e-12 ||T||) are computed together by the cluster's first
// workgroup; `zwork` (b x b, real) holds the cluster's finished vectors for
// the Gram-Schmidt steps.  Output column c = b - 1 - j (descending order).
template <int kPL>
__global__ void __launch_bounds__(64) k_tri_vector(const double* __restrict__ d,
                                                   const double* __restrict__ e,
                                                   const double* __restrict__ lam, int b,
                                                   const double2* __restrict__ refl,
                                                   const double2* __restrict__ tau,
                                                   double* __restrict__ zwork,
                                                   double2* __restrict__ U,
                                                   double* __restrict__ theta) {
  constexpr int kN = 64 * kPL;
  __shared__ double sd[kN], se[kN], sl[kN], z[kN];
  __shared__ double w0[kN], w1[kN], w2[kN], w3[kN];
  __shared__ int sw[kN];
  __shared__ int bad;
  const int t = threadIdx.x, j = blockIdx.x;
  double emax2 = 0.0;
  for (int i = t; i < b; i += 64) {
    sd[i] = d[i];
    const double ei = i + 1 < b ? e[i] : 0.0;
    se[i] = ei;
    emax2 = fmax(emax2, ei * ei);
    sl[i] = lam[i];
  }
  emax2 = wave_max(emax2);
  __syncthreads();
  const double nrm = fmax(fabs(sl[0]), fabs(sl[b - 1]));
  const double pivmin = DBL_MIN * fmax(1.0, emax2);
  const double ctol = 1e-12 * nrm;
  int cs = j, ce = j;
  while (cs > 0 && sl[cs] - sl[cs - 1] <= ctol) --cs;
  while (ce + 1 < b && sl[ce + 1] - sl[ce] <= ctol) ++ce;
  if (cs != j) return;  // the cluster's first workgroup computes it
  bool inverse = ce > cs;
  if (!inverse) {
    twisted_vector_wave(sd, se, b, sl[j], pivmin, w0, w1, w2, w3, z);
    // residual ||(T - lambda) z||_inf against a few ulps of ||T||
    const double lj = sl[j];
    double r = 0.0;
    for (int i = t; i < b; i += 64) {
      double v = (sd[i] - lj) * z[i];
      if (i > 0) v += se[i - 1] * z[i - 1];
      if (i + 1 < b) v += se[i] * z[i + 1];
      r = fmax(r, fabs(v));
    }
    r = wave_max(r);
    if (t == 0) bad = !(r <= 1e3 * b * DBL_EPSILON * nrm + pivmin);
    __syncthreads();
    inverse = bad != 0;
    if (!inverse) {
      if (t == 0) theta[b - 1 - j] = sl[j];
      back_transform<kPL>(z, b, refl, tau, U, b - 1 - j);
      return;
    }
  }
  const double tiny = fmax(DBL_EPSILON * nrm, pivmin);
  for (int q = cs; q <= ce; ++q) {
    for (int i = t; i < b; i += 64) z[i] = tri::start_value(q, i);
    if (t == 0) tri::lu_factor(sd, se, b, sl[q], tiny, w0, w1, w2, w3, sw);
    __syncthreads();
    for (int it = 0; it < 3; ++it) {
      if (t == 0) tri::lu_solve(b, w0, w1, w2, w3, sw, z);
      __syncthreads();
      // classical Gram-Schmidt against the finished members, twice
      for (int pass = 0; pass < 2; ++pass) {
        for (int p = cs; p < q; ++p) {
          const double* zp = zwork + size_t(p) * b;
          double s = 0.0;
          for (int i = t; i < b; i += 64) s += zp[i] * z[i];
          s = wave_sum(s);
          for (int i = t; i < b; i += 64) z[i] -= s * zp[i];
          __syncthreads();
        }
      }
      wave_normalize(z, b);
    }
    for (int i = t; i < b; i += 64) zwork[size_t(q) * b + i] = z[i];
    __threadfence_block();
    if (t == 0) theta[b - 1 - q] = sl[q];
    back_transform<kPL>(z, b, refl, tau, U, b - 1 - q);
    __syncthreads();
  }
}

}  // namespace

// Eigen-decomposition H = U diag(theta) U^H of the b x b Hermitian matrix H
// (column-major), eigenvalues descending.  ws must hold
// heev_workspace_doubles(b) doubles.
size_t heev_workspace_doubles(int b) {
  const size_t bb = size_t(b) * b;
  // refl (complex b*b), two reduction matrices for orders above 128 (complex
  // b*b each), zwork (b*b), tau (complex b), d, e, lam (b each), the
  // product vectors of the stepped reduction (two complex b)
  return 2 * bb + 4 * bb + bb + 2 * size_t(b) + 3 * size_t(b) + 4 * size_t(b) + 64;
}

pisco_status_t run_heev(Handle* h, const double2* H, int b, double2* U, double* theta,
                        double* ws) {
  if (b < 1 || b > kTriMax) {
    h->last_error = "heev: order out of range";
    return PISCO_ERR_UNSUPPORTED;
  }
  const size_t bb = size_t(b) * b;
  double2* refl = reinterpret_cast<double2*>(ws);
  double2* gwork = refl + bb;
  double* zwork = reinterpret_cast<double*>(gwork + bb);
  double2* tau = reinterpret_cast<double2*>(zwork + bb);
  double* d = reinterpret_cast<double*>(tau + b);
  double* e = d + b;
  double* lam = e + b;
  double2* gwork2 = reinterpret_cast<double2*>(lam + b);
  double2* xvec = gwork2 + bb;
  if (b <= kTrdLdsMax)
    PISCO_KERNEL(h, k_hetrd_reg<kTrdLdsMax / 8>, dim3(1), dim3(1024), 0, H, b, refl, tau, d, e);
  else if (b <= 128)
    PISCO_KERNEL(h, k_hetrd_reg<16>, dim3(1), dim3(1024), 0, H, b, refl, tau, d, e);
  else {
    // one launch per step on many one-wave workgroups, the matrix alternating
    // between two buffers
    PISCO_KERNEL(h, k_hetrd_sym, dim3(ceil_div(bb, 256)), dim3(256), 0, H, b, gwork);
    for (int k = 0; k < b; ++k) {
      const int m = b - 1 - k;
      const unsigned g = m > 1 ? unsigned(m) : 1u;
      const double2* rd = k == 0 ? gwork : ((k - 1) & 1 ? gwork2 : gwork);
      double2* wr = (k & 1) ? gwork2 : gwork;
      // x_{k-1} is read by every workgroup while x_k is written: two vectors
      const double2* xin = (k & 1) ? xvec : xvec + b;
      double2* xout = (k & 1) ? xvec + b : xvec;
      if (b <= 256)
        PISCO_KERNEL(h, k_hetrd_step<4>, dim3(g), dim3(64), 0, rd, wr, b, k, xin, xout, refl,
                     tau, d, e);
      else if (b <= 384)
        PISCO_KERNEL(h, k_hetrd_step<6>, dim3(g), dim3(64), 0, rd, wr, b, k, xin, xout, refl,
                     tau, d, e);
      else if (b <= 512)
        PISCO_KERNEL(h, k_hetrd_step<8>, dim3(g), dim3(64), 0, rd, wr, b, k, xin, xout, refl,
                     tau, d, e);
      else
        PISCO_KERNEL(h, k_hetrd_step<16>, dim3(g), dim3(64), 0, rd, wr, b, k, xin, xout, refl,
                     tau, d, e);
    }
  }
  PISCO_KERNEL(h, k_tri_eigval, dim3(b), dim3(kEigThreads), 0, d, e, b, lam);
  if (b <= 128)
    PISCO_KERNEL(h, k_tri_vector<2>, dim3(b), dim3(64), 0, d, e, lam, b, refl, tau, zwork, U, theta);
  else if (b <= 256)
    PISCO_KERNEL(h, k_tri_vector<4>, dim3(b), dim3(64), 0, d, e, lam, b, refl, tau, zwork, U, theta);
  else if (b <= 512)
    PISCO_KERNEL(h, k_tri_vector<8>, dim3(b), dim3(64), 0, d, e, lam, b, refl, tau, zwork, U, theta);
  else
    PISCO_KERNEL(h, k_tri_vector<16>, dim3(b), dim3(64), 0, d, e, lam, b, refl, tau, zwork, U, theta);
  return PISCO_OK;
}

}  // namespace pisco
