// Per-voxel G(x) on the low-resolution grid (Sec. IV-C, Eqs. 23-26).
//
// The paper forms W = sum_r h_r h_r^H over the null filters, sums its block
// diagonals into the lag kernel K_pq[m] (Eq. 26) and evaluates
// G_pq(x) = sum_m K_pq[m] e^{-i 2 pi m.x} with a zero-padded FFT.  Here the
// same K is obtained from the signal vectors v_r (complement route, Eq. 20):
//   K_pq = |Lambda| delta_pq delta[m] - K^s_pq,
//   K^s_pq[m] = sum_r sum_s conj(v_r[n_s + m, p]) v_r[n_s, q],
// and the correlation over s is done in the frequency domain, as the paper
// does for C^H C (Sec. IV-A):
//   1. filter spectra  F_r(f, q) = sum_{n in Lambda} v_r[n, q] e^{+i 2 pi n.f/Lk}
//      on a grid of Lk = 4 tau + 1 points per dimension (separable passes);
//   2. K^s_hat(f)_pq = sum_r conj(F_r(f, p)) F_r(f, q)   (contraction over r);
//   3. K^s[m] = (1/Lk^D) sum_f K^s_hat(f) e^{+i 2 pi m.f/Lk}, |m_d| <= 2 tau;
//   4. G^s(x) = sum_m K^s[m] e^{-i 2 pi m.x} on the low-res grid and
//      G = |Lambda| I - G^s.
// Lk = 4 tau + 1 is the smallest grid that holds every lag without aliasing.
#include <cmath>

#include <cstdio>

#include "common.hpp"

namespace pisco {

// box[r][q][cell] = v_r[q|Lambda| + i(cell)] for r < r_s, else 0 (FP64 -> FP32)
__global__ void k_scatter_box(const double2* __restrict__ basis,
                              const int32_t* __restrict__ counts, const int* __restrict__ map,
                              float2* __restrict__ box, int n, int L, int Q, int b,
                              int ncell) {
  const long long idx = blockIdx.x * 256LL + threadIdx.x;
  if (idx >= 1LL * b * Q * ncell) return;
  const int cell = int(idx % ncell);
  const long long rq = idx / ncell;
  const int q = int(rq % Q), r = int(rq / Q);
  const int rs = counts[0];
  const int i = map[cell];
  float2 v = make_float2(0.f, 0.f);
  if (i >= 0 && r < rs) {
    const double2 d = basis[size_t(r) * n + size_t(q) * L + i];
    v = make_float2(float(d.x), float(d.y));
  }
  box[idx] = v;
}

// Filter spectra in one pass per (r, q) workgroup: the box of v_r's channel
// q gathered from the basis (FP64 -> FP32), then the x, y and z DFTs of the
// separable zero-padded transform (box -> K = 2 box - 1 per axis, M1 tables)
// in LDS, the spectrum written once: Fh[r][q][fz][fy][fx].  Only rows r < r_s
// are formed (the contraction reads no others).  Each pass gives a thread one
// line of the box (its inputs in registers) and a range of frequencies that
// is the same across the wave, so a table row is one batch of wave-uniform
// (scalar) loads.  LDS: region A holds the box and later the y result,
// region B the x result.  kBox is the box edge, k3D whether z is transformed.
__device__ inline float2 cfma(float2 m, float2 v, float2 acc) {
  acc.x = fmaf(m.x, v.x, fmaf(-m.y, v.y, acc.x));
  acc.y = fmaf(m.x, v.y, fmaf(m.y, v.x, acc.y));
  return acc;
}

template <int kBox>
__device__ inline float2 dft_row(const float2* __restrict__ Mrow, const float2 (&v)[kBox]) {
  float2 acc = make_float2(0.f, 0.f);
#pragma unroll
  for (int i = 0; i < kBox; ++i) acc = cfma(Mrow[i], v[i], acc);
  return acc;
}

template <int kBox, bool k3D>
__global__ void __launch_bounds__(256) k_filter_spectra(
    const double2* __restrict__ basis, const int32_t* __restrict__ counts,
    const int* __restrict__ map, const float2* __restrict__ Mx, const float2* __restrict__ My,
    const float2* __restrict__ Mz, float2* __restrict__ Fh, int n, int L, int Q) {
  constexpr int K = 2 * kBox - 1, Bz = k3D ? kBox : 1, Kz = k3D ? K : 1;
  constexpr int kCells = Bz * kBox * kBox, kPlane = K * K;
  constexpr int kRegionA = kCells > Bz * kPlane ? kCells : Bz * kPlane;
  extern __shared__ float2 sm[];
  const int rq = blockIdx.x, r = rq / Q, q = rq - r * Q;
  if (r >= counts[0]) return;
  const int tid = threadIdx.x;
  float2* bx = sm;             // [Bz][box][box]
  float2* t2 = sm;             // [Bz][K][K] (after the x pass)
  float2* t1 = sm + kRegionA;  // [Bz][box][K]
  const double2* v_r = basis + size_t(r) * n + size_t(q) * L;
  for (int cell = tid; cell < kCells; cell += 256) {
    const int i = map[cell];
    float2 v = make_float2(0.f, 0.f);
    if (i >= 0) {
      const double2 d = v_r[i];
      v = make_float2(float(d.x), float(d.y));
    }
    bx[cell] = v;
  }
  __syncthreads();
  float2 v[kBox];
  // x: row (cz, cy) of the box; threads 0-127 take the lower frequencies,
  // 128-255 the upper ones (wave-uniform halves)
  {
    constexpr int kRows = Bz * kBox, kHalf = (K + 1) / 2;
    const int half = tid >> 7, f0 = half ? kHalf : 0, f1 = half ? K : kHalf;
    for (int row = tid & 127; row < kRows; row += 128) {
#pragma unroll
      for (int i = 0; i < kBox; ++i) v[i] = bx[row * kBox + i];
      for (int f = f0; f < f1; ++f) t1[row * K + f] = dft_row<kBox>(Mx + f * kBox, v);
    }
  }
  __syncthreads();
  // y: (cz, fx) -> K frequencies
  for (int e = tid; e < Bz * K; e += 256) {
    const int cz = e / K, fx = e - cz * K;
#pragma unroll
    for (int i = 0; i < kBox; ++i) v[i] = t1[(cz * kBox + i) * K + fx];
    for (int f = 0; f < K; ++f) t2[(cz * K + f) * K + fx] = dft_row<kBox>(My + f * kBox, v);
  }
  __syncthreads();
  // z: (fy, fx) -> Kz frequencies, straight to the spectrum
  float2* dst = Fh + size_t(rq) * Kz * kPlane;
  for (int e = tid; e < kPlane; e += 256) {
    if (!k3D) {
      dst[e] = t2[e];
      continue;
    }
#pragma unroll
    for (int i = 0; i < kBox; ++i) v[i] = t2[i * kPlane + e];
    for (int f = 0; f < Kz; ++f) dst[size_t(f) * kPlane + e] = dft_row<kBox>(Mz + f * kBox, v);
  }
}

template <int kBox>
static size_t filter_spectra_lds(bool d3) {
  const size_t K = 2 * kBox - 1, Bz = d3 ? kBox : 1;
  const size_t cells = Bz * kBox * kBox, a = cells > Bz * K * K ? cells : Bz * K * K;
  return (a + Bz * kBox * K) * sizeof(float2);
}

// The one-pass filter spectra where the box edge has an instance and the LDS
// fits in 64 KB; PISCO_ERR_UNSUPPORTED (nothing launched) otherwise.
static pisco_status_t filter_spectra(Handle* h, const Plan& p, int b, const double2* basis,
                                     const int32_t* counts, const int* map, const Tables& t,
                                     float2* Fh) {
  const int box = 2 * p.tau + 1;
  const bool d3 = p.D == 3;
  if (p.K[2] != 2 * box - 1 || p.K[1] != 2 * box - 1 || (d3 && p.K[0] != 2 * box - 1))
    return PISCO_ERR_UNSUPPORTED;
  const float2* Mz = d3 ? t.M1[0] : t.M1[1];
  const dim3 grid(unsigned(b * p.Q));
#define PISCO_FS_CASE(B)                                                                     \
  case B: {                                                                                  \
    const size_t lds = filter_spectra_lds<B>(d3);                                            \
    if (lds > 65536) return PISCO_ERR_UNSUPPORTED;                                           \
    if (d3)                                                                                  \
      PISCO_KERNEL(h, (k_filter_spectra<B, true>), grid, dim3(256), lds, basis, counts, map, \
                   t.M1[2], t.M1[1], Mz, Fh, p.n, p.L, p.Q);                                 \
    else                                                                                     \
      PISCO_KERNEL(h, (k_filter_spectra<B, false>), grid, dim3(256), lds, basis, counts,    \
                   map, t.M1[2], t.M1[1], Mz, Fh, p.n, p.L, p.Q);                            \
    return PISCO_OK;                                                                         \
  }
  switch (box) {
    PISCO_FS_CASE(5)
    PISCO_FS_CASE(7)
    PISCO_FS_CASE(9)
    PISCO_FS_CASE(11)
    PISCO_FS_CASE(13)
    default: return PISCO_ERR_UNSUPPORTED;
  }
#undef PISCO_FS_CASE
}

// Kh[pair(p,q)][f] = sum_{r < r_s} conj(F[r][p][f]) F[r][q][f]
// Block: FT frequencies x Q channels; r staged through LDS in chunks of 8.
__global__ void __launch_bounds__(256) k_herk(const float2* __restrict__ F,
                                              const int32_t* __restrict__ counts,
                                              float2* __restrict__ Kh, int Q, int nK, int FT) {
  __shared__ float2 tile[8 * 256];
  const int t = threadIdx.x;
  const int fl = t % FT, q = t / FT;
  // XCD-contiguous frequency blocks: the blocks that share a 128-byte line
  // of F run on one XCD (one L2)
  const int fb = int(xcd_block(blockIdx.x, gridDim.x));
  const int f = fb * FT + fl;
  const bool active = q < Q && f < nK;
  const int rs = counts[0];
  float2 acc[kMaxQ];
#pragma unroll
  for (int p = 0; p < kMaxQ; ++p) acc[p] = make_float2(0.f, 0.f);
  for (int r0 = 0; r0 < rs; r0 += 8) {
    const int rc = rs - r0 < 8 ? rs - r0 : 8;
    for (int e = t; e < rc * Q * FT; e += 256) {
      const int rr = e / (Q * FT), rem = e - rr * Q * FT, qq = rem / FT, ff = rem - qq * FT;
      const int gf = fb * FT + ff;
      tile[e] = gf < nK ? F[(size_t(r0 + rr) * Q + qq) * nK + gf] : make_float2(0.f, 0.f);
    }
    __syncthreads();
    if (active) {
      for (int rr = 0; rr < rc; ++rr) {
        const float2* row = tile + rr * Q * FT;
        const float2 x = row[q * FT + fl];
#pragma unroll
        for (int p = 0; p < kMaxQ; ++p)
          if (p <= q) {
            const float2 y = row[p * FT + fl];
            acc[p].x = fmaf(y.x, x.x, fmaf(y.y, x.y, acc[p].x));
            acc[p].y = fmaf(y.x, x.y, fmaf(-y.y, x.x, acc[p].y));
          }
      }
    }
    __syncthreads();
  }
  if (!active) return;
#pragma unroll
  for (int p = 0; p < kMaxQ; ++p)
    if (p <= q) {
      const int pair = p * Q - p * (p - 1) / 2 + (q - p);
      Kh[size_t(pair) * nK + f] = acc[p];
    }
}

// Split-precision variant of k_herk on the matrix cores (FP32 accumulation).
// kPrec = PISCO_PREC_SPLIT_F16: each FP32 operand x, scaled by 2^e so that
// FP16's range is used, is split into x_hi = fp16(x) and x_lo = fp16(x -
// x_hi) and a product is x_hi y_hi + x_hi y_lo + x_lo y_hi (three MFMAs; the
// dropped x_lo y_lo is below 2^-22 relative).  kPrec = PISCO_PREC_SPLIT_BF16:
// three BF16 parts hi, mid, lo and the six cross products of total order
// <= 2.  Workgroup: 4 frequencies, one per wave; r runs in chunks of 32
// staged in LDS as [r][q][f] (f padded to 5 against bank conflicts).  For one frequency the Q x Q result is C = A^H A with A the
// r x Q matrix F[.][.][f]: Re C = Ar^T Ar + Ai^T Ai, Im C = Ar^T Ai - Ai^T Ar,
// as 16 x 16 x 32 blocks on gfx950's double-K shapes (upper blocks only).
// Operand lanes: lane l holds row (column) l % 16 at k = 8 (l / 16) + j,
// j < 8 (the same for both operands); accumulator element v of lane l is
// row 4 (l / 16) + v, column l % 16.
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef short bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ inline short bf16_rne(float f) {
  unsigned u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return short(u >> 16);
}
__device__ inline float bf16_to_f32(short h) {
  return __uint_as_float(static_cast<unsigned>(static_cast<unsigned short>(h)) << 16);
}

template <int kPrec>
struct SplitOps;

template <>
struct SplitOps<PISCO_PREC_SPLIT_F16> {
  static constexpr int kParts = 2;
  typedef f16x8 vec;
  __device__ static void split(const float (&x)[8], float s, vec (&out)[kParts]) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const float v = x[j] * s;
      const _Float16 hi = static_cast<_Float16>(v);
      out[0][j] = hi;
      out[1][j] = static_cast<_Float16>(v - static_cast<float>(hi));
    }
  }
  __device__ static vec neg(vec a) { return -a; }
  __device__ static f32x4 mma(vec a, vec b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
  // (part of x, part of y) pairs kept: hi hi, hi lo, lo hi
  static constexpr int kTerms = 3;
  __device__ static constexpr int ta(int i) { return i == 2 ? 1 : 0; }
  __device__ static constexpr int tb(int i) { return i == 1 ? 1 : 0; }
};

template <>
struct SplitOps<PISCO_PREC_SPLIT_BF16> {
  static constexpr int kParts = 3;
  typedef bf16x8 vec;
  __device__ static void split(const float (&x)[8], float, vec (&out)[kParts]) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      float v = x[j];
      const short hi = bf16_rne(v);
      v -= bf16_to_f32(hi);
      const short mid = bf16_rne(v);
      v -= bf16_to_f32(mid);
      out[0][j] = hi;
      out[1][j] = mid;
      out[2][j] = bf16_rne(v);
    }
  }
  __device__ static vec neg(vec a) { return a ^ short(0x8000); }
  __device__ static f32x4 mma(vec a, vec b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, a),
                                                   __builtin_bit_cast(bf16x8_t, b), c, 0, 0, 0);
  }
  // hi hi, hi mid, mid hi, hi lo, lo hi, mid mid
  static constexpr int kTerms = 6;
  __device__ static constexpr int ta(int i) { return i == 2 ? 1 : (i == 4 ? 2 : (i == 5 ? 1 : 0)); }
  __device__ static constexpr int tb(int i) { return i == 1 ? 1 : (i == 3 ? 2 : (i == 5 ? 1 : 0)); }
};

template <int kPrec>
__global__ void __launch_bounds__(256) k_herk_mfma(const float2* __restrict__ F,
                                                   const int32_t* __restrict__ counts,
                                                   float2* __restrict__ Kh, int Q, int nK,
                                                   float scale) {
  using Ops = SplitOps<kPrec>;
  using vec = typename Ops::vec;
  constexpr int kFB = 4, kFP = 5, kFW = 1;  // frequencies per block / padded / per wave
  constexpr int kR = 32;  // r per chunk (the MFMA's K)
  __shared__ float2 tile[kR * kMaxQ * kFP];
  const int t = threadIdx.x, wv = t >> 6, l = t & 63;
  const int li = l & 15, kg = l >> 4;
  // XCD-contiguous frequency blocks: the four blocks that share a 128-byte
  // line of F run on one XCD (one L2), so the line is fetched once
  const int f0 = int(xcd_block(blockIdx.x, gridDim.x)) * kFB;
  const int rs = counts[0];
  const int nqb = Q > 16 ? 2 : 1;
  f32x4 cr[kFW][3], ci[kFW][3];
#pragma unroll
  for (int fi = 0; fi < kFW; ++fi)
#pragma unroll
    for (int bk = 0; bk < 3; ++bk) {
      cr[fi][bk] = f32x4{0.f, 0.f, 0.f, 0.f};
      ci[fi][bk] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
  for (int r0 = 0; r0 < rs; r0 += kR) {
    for (int e = t; e < kR * Q * kFB; e += 256) {
      const int ff = e % kFB, rq = e / kFB, rr = rq / Q;
      const int f = f0 + ff;
      tile[rq * kFP + ff] = (r0 + rr < rs && f < nK) ? F[size_t(r0 * Q + rq) * nK + f]
                                                     : make_float2(0.f, 0.f);
    }
    __syncthreads();
#pragma unroll
    for (int fi = 0; fi < kFW; ++fi) {
      const int ff = wv * kFW + fi;
      // parts of Re and Im for the lane's column in channel block 0 and 1
      vec re[2][Ops::kParts], im[2][Ops::kParts];
#pragma unroll
      for (int cb = 0; cb < 2; ++cb) {
        float xr[8], xi[8];
        const int q = 16 * cb + li;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const float2 v = q < Q ? tile[((8 * kg + j) * Q + q) * kFP + ff] : make_float2(0.f, 0.f);
          xr[j] = v.x;
          xi[j] = v.y;
        }
        Ops::split(xr, scale, re[cb]);
        Ops::split(xi, scale, im[cb]);
      }
#pragma unroll
      for (int bk = 0; bk < 3; ++bk) {
        const int pb = bk == 2 ? 1 : 0, qb = bk == 0 ? 0 : 1;
        if (qb >= nqb) continue;
#pragma unroll
        for (int term = 0; term < Ops::kTerms; ++term) {
          const vec arp = re[pb][Ops::ta(term)], aip = im[pb][Ops::ta(term)];
          const vec brq = re[qb][Ops::tb(term)], biq = im[qb][Ops::tb(term)];
          cr[fi][bk] = Ops::mma(arp, brq, cr[fi][bk]);
          cr[fi][bk] = Ops::mma(aip, biq, cr[fi][bk]);
          ci[fi][bk] = Ops::mma(arp, biq, ci[fi][bk]);
          ci[fi][bk] = Ops::mma(Ops::neg(aip), brq, ci[fi][bk]);
        }
      }
    }
    __syncthreads();
  }
  const float inv = kPrec == PISCO_PREC_SPLIT_F16 ? 1.f / (scale * scale) : 1.f;
#pragma unroll
  for (int fi = 0; fi < kFW; ++fi) {
    const int f = f0 + wv * kFW + fi;
    if (f >= nK) continue;
#pragma unroll
    for (int bk = 0; bk < 3; ++bk) {
      const int pb = bk == 2 ? 1 : 0, qb = bk == 0 ? 0 : 1;
      if (qb >= nqb) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int p = 16 * pb + 4 * kg + v, q = 16 * qb + li;
        if (p <= q && q < Q) {
          const int pair = p * Q - p * (p - 1) / 2 + (q - p);
          Kh[size_t(pair) * nK + f] = make_float2(cr[fi][bk][v] * inv, ci[fi][bk][v] * inv);
        }
      }
    }
  }
}

// G = |Lambda| I - G^s on the packed planes; diagonal entries real.
__global__ void k_gx_finish(float2* __restrict__ G, int Q, long long N, float bound) {
  const long long idx = blockIdx.x * 256LL + threadIdx.x;
  const int P = Q * (Q + 1) / 2;
  if (idx >= 1LL * P * N) return;
  const int pair = int(idx / N);
  // pair is diagonal when it is the first entry of its row block
  int p = 0, base = 0;
  while (pair >= base + (Q - p)) {
    base += Q - p;
    ++p;
  }
  const bool diag = pair == base;
  const float2 g = G[idx];
  G[idx] = diag ? make_float2(bound - g.x, 0.f) : make_float2(-g.x, -g.y);
}

static pisco_status_t chain(Handle* h, const float2* in, float2* out, int shape[4],
                            int axis, int nout, const float2* M) {
  pisco_status_t st = axis_transform(h, in, out, shape, axis, nout, M);
  shape[axis] = nout;
  return st;
}

pisco_status_t run_gx(Handle* h, const Plan& p, const Tables& t, int b, int precision,
                      const double2* basis, const int32_t* counts, float2* G, void* ws) {
  GxWs w;
  layout_gx(p, b, ws, &w);
  const int Q = p.Q, tau = p.tau, P = p.P;
  const int box = 2 * tau + 1;
  const int Bz = p.D == 3 ? box : 1;
  const int ncell = Bz * box * box;
  pisco_status_t st;
  const float2* const* M1 = t.M1;
  const float2* const* M4 = t.M4;
  const int* map = t.boxmap;
  float2* bufA = w.Tmp;
  float2* bufB = w.Tmp + w.tmp_half;
  // 1. filter spectra: [bQ][Bz][box][box] -> [bQ][Kz][Ky][Kx] (ends in Fh);
  // one pass per (r, q) where the box edge has an instance and fits
  st = filter_spectra(h, p, b, basis, counts, map, t, w.Fh);
  if (st == PISCO_ERR_UNSUPPORTED) {
    PISCO_KERNEL(h, k_scatter_box, dim3(ceil_div(1LL * b * Q * ncell, 256)), dim3(256), 0, basis, counts, map, bufA, p.n, p.L, Q, b, ncell);
    int shp[4] = {b * Q, Bz, box, box};
    if (p.D == 3) {
      if ((st = chain(h, bufA, bufB, shp, 3, p.K[2], M1[2]))) return st;
      if ((st = chain(h, bufB, bufA, shp, 2, p.K[1], M1[1]))) return st;
      if ((st = chain(h, bufA, w.Fh, shp, 1, p.K[0], M1[0]))) return st;
    } else {
      if ((st = chain(h, bufA, bufB, shp, 3, p.K[2], M1[2]))) return st;
      if ((st = chain(h, bufB, w.Fh, shp, 2, p.K[1], M1[1]))) return st;
    }
  } else if (st) {
    return st;
  }
  // 2. contraction over the signal vectors
  if (precision == PISCO_PREC_SPLIT_F16) {
    // |F_r(f, q)| <= sum_n |v_r[n, q]| <= sqrt(|Lambda|) for unit v_r: scale
    // so that this bound maps below 2^15 (FP16 holds up to 65504)
    const float scale = std::ldexp(1.f, int(std::floor(15.0 - 0.5 * std::log2(double(p.L)))));
    PISCO_KERNEL(h, k_herk_mfma<PISCO_PREC_SPLIT_F16>, dim3(ceil_div(p.nK, 4)), dim3(256), 0, w.Fh, counts, w.Kh, Q, p.nK, scale);
  } else if (precision == PISCO_PREC_SPLIT_BF16) {
    PISCO_KERNEL(h, k_herk_mfma<PISCO_PREC_SPLIT_BF16>, dim3(ceil_div(p.nK, 4)), dim3(256), 0, w.Fh, counts, w.Kh, Q, p.nK, 1.f);
  } else {
    const int FT = 256 / Q;
    PISCO_KERNEL(h, k_herk, dim3(ceil_div(p.nK, FT)), dim3(256), 0, w.Fh, counts, w.Kh, Q, p.nK, FT);
  }
  // 3. evaluate on the low-res grid straight from the spectra (the lags and
  // their evaluation composed per axis in the M4 tables):
  // [P][Kz][Ky][Kx] -> [P][lr0][lr1][lr2]
  // (the last pass stores G = |Lambda| I - G^s where it runs on the matrix
  // cores; otherwise a pass of its own does)
  int shl[4] = {P, p.K[0], p.K[1], p.K[2]};
  const float bound = float(p.L);
  const float2* last_in = nullptr;
  int last_axis = 0;
  if (p.D == 3) {
    if ((st = chain(h, w.Kh, bufA, shl, 3, p.lr[2], M4[2]))) return st;
    if ((st = chain(h, bufA, bufB, shl, 2, p.lr[1], M4[1]))) return st;
    last_in = bufB;
    last_axis = 1;
  } else {
    if ((st = chain(h, w.Kh, bufA, shl, 3, p.lr[2], M4[2]))) return st;
    last_in = bufA;
    last_axis = 2;
  }
  const int last = last_axis - 1;  // grid dimension of the last pass
  st = axis_transform_gx(h, last_in, G, shl, last_axis, p.lr[last], M4[last], Q, bound);
  if (st == PISCO_ERR_UNSUPPORTED) {
    if ((st = axis_transform(h, last_in, G, shl, last_axis, p.lr[last], M4[last]))) return st;
    PISCO_KERNEL(h, k_gx_finish, dim3(ceil_div(1LL * P * p.Nlr, 256)), dim3(256), 0, G, Q, p.Nlr,
                 bound);
  } else if (st) {
    return st;
  }
  return PISCO_OK;
}

}  // namespace pisco
