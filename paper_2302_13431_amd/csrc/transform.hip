// Separable small-matrix transforms along one axis of a batched 3D array, and
// the device-side builders of the matrices they apply (DFT, apodized DFT,
// periodic sinc interpolation).  Every multi-dimensional transform of the path
// outside the Gram FFTs (filter spectra, lag kernel, G(x) evaluation, the
// apodized low-resolution image and the interpolation) is a product of such
// one-axis passes.
#include <cmath>

#include <cstdio>

#include "common.hpp"

namespace pisco {

typedef float f32x4 __attribute__((ext_vector_type(4)));

// Element helpers: loads widen to the accumulation type T of the output.
template <class T> struct Acc;
template <> struct Acc<float2> {
  using S = float;
  __device__ static float2 zero() { return make_float2(0.f, 0.f); }
};
template <> struct Acc<double2> {
  using S = double;
  __device__ static double2 zero() { return make_double2(0.0, 0.0); }
};
template <class T, class U> __device__ inline T widen(U v) { return T{v.x, v.y}; }

// out[outer][o][inner] = sum_i M[o][i] in[outer][i][inner]   (inner > 1)
// Block = 256 consecutive (outer, inner) columns x a tile of kOT outputs;
// the tile's rows of M are staged in LDS and read as broadcasts, each input
// load feeds kOT complex multiply-adds.  kOT = 4 is used when 16 would leave
// the launch with too few workgroups to fill the chip.
constexpr int kMidMaxIn = 256;

// dst[e] = widen(src[e]) for e < n by a workgroup of 256 threads, four
// loads per thread in flight at once
template <class TO, class TI>
__device__ inline void stage_rows(TO* dst, const TI* __restrict__ src, int n) {
  int e0 = threadIdx.x;
  for (; e0 + 3 * 256 < n; e0 += 4 * 256) {
    TI v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = src[e0 + u * 256];
#pragma unroll
    for (int u = 0; u < 4; ++u) dst[e0 + u * 256] = widen<TO>(v[u]);
  }
  for (; e0 < n; e0 += 256) dst[e0] = widen<TO>(src[e0]);
}

template <class TI, class TO, int kOT>
__global__ void __launch_bounds__(256) k_axis_mid(const TI* __restrict__ in,
                                                  TO* __restrict__ out,
                                                  const TO* __restrict__ M, long long outer,
                                                  int nin, int nout, int inner) {
  __shared__ TO Ms[kOT * kMidMaxIn];
  const int o0 = blockIdx.y * kOT;
  const int cnt = nout - o0 < kOT ? nout - o0 : kOT;
  stage_rows(Ms, M + size_t(o0) * nin, cnt * nin);
  __syncthreads();
  const long long col = blockIdx.x * 256LL + threadIdx.x;
  if (col >= outer * inner) return;
  const long long ou = col / inner;
  const int ii = int(col - ou * inner);
  const TI* src = in + size_t(ou) * nin * inner + ii;
  TO* dst = out + size_t(ou) * nout * inner + ii;
  TO acc[kOT];
#pragma unroll
  for (int k = 0; k < kOT; ++k) acc[k] = Acc<TO>::zero();
  // inputs eight at a time, all eight loads in flight before the first is
  // used (one load per step would wait for each in turn)
  auto step = [&](const TO& x, int i) {
#pragma unroll
    for (int k = 0; k < kOT; ++k) {
      const TO m = Ms[k * nin + i];
      acc[k].x = fma(m.x, x.x, fma(-m.y, x.y, acc[k].x));
      acc[k].y = fma(m.x, x.y, fma(m.y, x.x, acc[k].y));
    }
  };
  int i = 0;
  for (; i + 8 <= nin; i += 8) {
    TO x[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) x[u] = widen<TO>(src[size_t(i + u) * inner]);
#pragma unroll
    for (int u = 0; u < 8; ++u) step(x[u], i + u);
  }
  for (; i < nin; ++i) step(widen<TO>(src[size_t(i) * inner]), i);
#pragma unroll
  for (int k = 0; k < kOT; ++k)
    if (k < cnt) dst[size_t(o0 + k) * inner] = acc[k];
}

// out[outer][o][inner] = sum_i M[o][i] in[outer][i][inner] for short
// transforms (nin <= NMAX): one thread per (outer, inner) column holds its
// nin inputs in registers (all loads in flight at once) and forms the nout
// outputs one after another; M is the same for every lane, so its entries
// come through scalar loads and no LDS is used.  FP64 output only.
template <class TI, int NMAX>
__global__ void __launch_bounds__(256) k_axis_reg(const TI* __restrict__ in,
                                                  double2* __restrict__ out,
                                                  const double2* __restrict__ M,
                                                  long long outer, int nin, int nout,
                                                  int inner) {
  const long long col = blockIdx.x * 256LL + threadIdx.x;
  if (col >= outer * inner) return;
  const long long ou = col / inner;
  const int ii = int(col - ou * inner);
  const TI* src = in + size_t(ou) * nin * inner + ii;
  double2* dst = out + size_t(ou) * nout * inner + ii;
  double2 x[NMAX];
#pragma unroll
  for (int i = 0; i < NMAX; ++i)
    x[i] = i < nin ? widen<double2>(src[size_t(i) * inner]) : make_double2(0.0, 0.0);
  for (int o = 0; o < nout; ++o) {
    const double2* m = M + size_t(o) * nin;
    double ar = 0.0, ai = 0.0;
#pragma unroll
    for (int i = 0; i < NMAX; ++i) {
      if (i < nin) {
        const double2 mv = m[i];
        ar = fma(mv.x, x[i].x, fma(-mv.y, x[i].y, ar));
        ai = fma(mv.x, x[i].y, fma(mv.y, x[i].x, ai));
      }
    }
    dst[size_t(o) * inner] = make_double2(ar, ai);
  }
}

// out[line][o] = sum_i M[o][i] in[line][i]   (contiguous lines)
// One output per thread: a block takes lpb = max(1, 256 / nout) lines,
// staged in LDS, so that even a long output line spreads over many
// workgroups; the rows of M come through the caches.
template <class TI, class TO>
__global__ void __launch_bounds__(256) k_axis_last(const TI* __restrict__ in,
                                                   TO* __restrict__ out,
                                                   const TO* __restrict__ M, long long lines,
                                                   int nin, int nout, int lpb) {
  using S = typename Acc<TO>::S;
  extern __shared__ unsigned char smem[];
  TO* sl = reinterpret_cast<TO*>(smem);  // [lpb][nin]
  const int per = (nout + 255) / 256;    // blocks per line when lpb == 1
  const long long l0 = per > 1 ? blockIdx.x / per : blockIdx.x * (long long)lpb;
  const int obase = per > 1 ? int(blockIdx.x % per) * 256 : 0;
  const int nl = per > 1 ? 1 : (lines - l0 < lpb ? int(lines - l0) : lpb);
  stage_rows(sl, in + size_t(l0) * nin, nl * nin);
  __syncthreads();
  const int span = per > 1 ? 256 : nout;
  const int ln = threadIdx.x / span, o = obase + threadIdx.x % span;
  if (ln >= nl || o >= nout) return;
  const TO* x = sl + ln * nin;
  const TO* m = M + size_t(o) * nin;
  S ar = 0, ai = 0;
  for (int i = 0; i < nin; ++i) {
    const TO mv = m[i], xv = x[i];
    ar = fma(mv.x, xv.x, fma(-mv.y, xv.y, ar));
    ai = fma(mv.x, xv.y, fma(mv.y, xv.x, ai));
  }
  out[size_t(l0 + ln) * nout + o] = TO{ar, ai};
}

// FP32 transforms on the matrix cores (v_mfma_f32_16x16x4f32, twice the
// FP32 vector rate without packed operations), for the passes with many
// outputs per input (the interpolation to the output grid, G(x) on the
// low-resolution grid).  A workgroup forms 64 x 64 tiles of the product
// C = M X over K = nin (rounded up to 4, zeros past nin) staged in LDS, four
// waves of 16 x 64.  A complex M takes the three-multiplication form (T1 =
// Ar Br, T2 = Ai Bi, T3 = (Ar + Ai)(Br + Bi); Re = T1 - T2, Im = T3 - T1 -
// T2); a real M (kReal: its imaginary parts are ignored) two products, Re =
// M Xr and Im = M Xi.  Operand lanes of the 16 x 16 x 4 shape: lane l
// supplies A row l % 16 and B column l % 16 at k = l / 16; accumulator
// element v of lane l is row 4 (l / 16) + v, column l % 16.
//   k_axis_mm_cols (inner > 1): X[k][col] = in[outer][k][inner0 + col],
//     A = M (64 outputs), B = X; the tile's outputs are written along inner.
//   k_axis_mm_lines (inner = 1): A = the lines' inputs (64 lines), B = M^T;
//     each line's 64 outputs are written along the line.
constexpr int kMmK = 64;  // nin at most (K padded to a multiple of 4)

// As[r][k] (row stride lda); Bs[k][c] (bt == false, stride ldb) or Bs[c][k].
// With kReal, M is A when bt == false (column tiles) and B when bt == true.
template <bool kReal>
__device__ inline void mm_tile(const float2* As, int lda, const float2* Bs, int ldb, bool bt,
                               int K4, f32x4 (&t1)[4], f32x4 (&t2)[4], f32x4 (&t3)[4]) {
  const int l = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int li = l & 15, kq = l >> 4;
#pragma unroll
  for (int j = 0; j < 4; ++j) t1[j] = t2[j] = t3[j] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < K4; k0 += 4) {
    const int k = k0 + kq;
    const float2 a = As[(16 * wv + li) * lda + k];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float2 b = bt ? Bs[(16 * j + li) * ldb + k] : Bs[k * ldb + 16 * j + li];
      if (!kReal) {
        t1[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b.x, t1[j], 0, 0, 0);
        t2[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, b.y, t2[j], 0, 0, 0);
        t3[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x + a.y, b.x + b.y, t3[j], 0, 0, 0);
      } else if (!bt) {  // A = M real
        t1[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b.x, t1[j], 0, 0, 0);
        t2[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b.y, t2[j], 0, 0, 0);
      } else {  // B = M^T real
        t1[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b.x, t1[j], 0, 0, 0);
        t2[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, b.x, t2[j], 0, 0, 0);
      }
    }
  }
}

template <bool kReal>
__device__ inline float2 mm_result(const f32x4& t1, const f32x4& t2, const f32x4& t3, int v) {
  return kReal ? make_float2(t1[v], t2[v]) : make_float2(t1[v] - t2[v], t3[v] - t1[v] - t2[v]);
}

// Ms[o][k] = M[o0 + o][k] (zeros past nout and nin), row stride kMmK + 1
__device__ inline void mm_stage_m(float2* Ms, const float2* __restrict__ M, int o0, int nout,
                                  int nin, int K4) {
  for (int e = threadIdx.x; e < 64 * K4; e += 256) {
    const int o = e / K4, k = e - o * K4;
    Ms[o * (kMmK + 1) + k] =
        o0 + o < nout && k < nin ? M[size_t(o0 + o) * nin + k] : make_float2(0.f, 0.f);
  }
}

// kMmTiles input tiles per workgroup, one after another: M staged once, the
// next tile's inputs loaded into registers while the current one is
// multiplied.  Both kernels take a 1-D grid whose logical workgroup index
// (XCD-contiguous) runs fastest over the 64-output tiles: the workgroups that
// read one input tile run together on one XCD, so the tile is fetched from
// HBM once.
constexpr int kMmTiles = 8;

// The input tiles of k_axis_mm_cols run over (outer index, 64 columns of
// inner) with the column tile fastest, so that a short inner axis still gives
// a workgroup kMmTiles tiles.
// kEpi = 1: the outer index is a packed Hermitian pair of a Q x Q matrix
// (row-major upper triangle) and the result y is stored as bound - Re y (a
// diagonal pair, imaginary part zero) or -y (off-diagonal): G = |Lambda| I -
// G^s without a pass of its own.
template <bool kReal, int kEpi>
__global__ void __launch_bounds__(256) k_axis_mm_cols(const float2* __restrict__ in,
                                                      float2* __restrict__ out,
                                                      const float2* __restrict__ M,
                                                      long long outer, int nin, int nout,
                                                      int inner, int epi_q, float epi_bound) {
  constexpr int XS = 64 + 1;  // Xs row stride
  constexpr int kPer = kMmK * 64 / 256;  // staged elements per thread
  __shared__ float2 Ms[64 * (kMmK + 1)];
  __shared__ float2 Xs[kMmK * XS];
  const int K4 = (nin + 3) & ~3;
  const int ctiles = (inner + 63) / 64;
  const long long tiles = outer * ctiles;
  const int otiles = (nout + 63) / 64;
  const long long lb = xcd_block(blockIdx.x, gridDim.x);
  const int o0 = int(lb % otiles) * 64;
  const long long tb = lb / otiles * kMmTiles;
  const long long te = tiles < tb + kMmTiles ? tiles : tb + kMmTiles;
  mm_stage_m(Ms, M, o0, nout, nin, K4);
  float2 x[kPer];
  auto load = [&](long long tile) {
    const long long ou = tile / ctiles;
    const int c0 = int(tile - ou * ctiles) * 64;
    const float2* src = in + size_t(ou) * nin * inner;
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int e = threadIdx.x + 256 * u, k = e >> 6, c = e & 63;
      x[u] = k < nin && c0 + c < inner ? src[size_t(k) * inner + c0 + c] : make_float2(0.f, 0.f);
    }
  };
  const int l = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (tb < te) load(tb);
  for (long long tile = tb; tile < te; ++tile) {
    __syncthreads();  // the previous tile's products are done with Xs
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int e = threadIdx.x + 256 * u, k = e >> 6, c = e & 63;
      if (k < K4) Xs[k * XS + c] = x[u];
    }
    __syncthreads();
    if (tile + 1 < te) load(tile + 1);
    f32x4 t1[4], t2[4], t3[4];
    mm_tile<kReal>(Ms, kMmK + 1, Xs, XS, false, K4, t1, t2, t3);
    const long long ou = tile / ctiles;
    const int c0 = int(tile - ou * ctiles) * 64;
    float2* dst = out + size_t(ou) * nout * inner;
    bool diag = false;
    if (kEpi == 1) {  // pair ou is diagonal when it opens its row's block
      long long base = 0;
      for (int p = 0; p < epi_q && base <= ou; base += epi_q - p, ++p) diag = diag || base == ou;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int o = o0 + 16 * wv + 4 * (l >> 4) + v, c = c0 + 16 * j + (l & 15);
        float2 y = mm_result<kReal>(t1[j], t2[j], t3[j], v);
        if (kEpi == 1) y = diag ? make_float2(epi_bound - y.x, 0.f) : make_float2(-y.x, -y.y);
        if (o < nout && c < inner) dst[size_t(o) * inner + c] = y;
      }
  }
}

template <bool kReal>
__global__ void __launch_bounds__(256) k_axis_mm_lines(const float2* __restrict__ in,
                                                       float2* __restrict__ out,
                                                       const float2* __restrict__ M,
                                                       long long lines, int nin, int nout) {
  constexpr int kPer = kMmK * 64 / 256;  // staged elements per thread
  __shared__ float2 Ms[64 * (kMmK + 1)];
  __shared__ float2 Xs[64 * (kMmK + 1)];
  const int K4 = (nin + 3) & ~3;
  const int otiles = (nout + 63) / 64;
  const long long tiles = (lines + 63) / 64;
  const long long lb = xcd_block(blockIdx.x, gridDim.x);
  const int o0 = int(lb % otiles) * 64;
  const long long tb = lb / otiles * kMmTiles;
  const long long te = tiles < tb + kMmTiles ? tiles : tb + kMmTiles;
  mm_stage_m(Ms, M, o0, nout, nin, K4);
  // element u of this thread: line r, input k of a 64-line tile (r < 64 for
  // e < 64 K4), at offset r nin + k from the tile's first line
  int off[kPer], lds[kPer];
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int e = threadIdx.x + 256 * u, r = e / K4, k = e - r * K4;
    const bool use = e < 64 * K4;
    lds[u] = use ? r * (kMmK + 1) + k : -1;
    off[u] = use && k < nin ? r * nin + k : -1;
  }
  float2 x[kPer];
  auto load = [&](long long tile) {
    const long long l0 = tile * 64;
    const float2* src = in + size_t(l0) * nin;
    const long long lim = (lines - l0) * nin;  // elements of this tile in range
#pragma unroll
    for (int u = 0; u < kPer; ++u)
      x[u] = off[u] >= 0 && off[u] < lim ? src[off[u]] : make_float2(0.f, 0.f);
  };
  const int l = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (tb < te) load(tb);
  for (long long tile = tb; tile < te; ++tile) {
    __syncthreads();  // the previous tile's products are done with Xs
#pragma unroll
    for (int u = 0; u < kPer; ++u)
      if (lds[u] >= 0) Xs[lds[u]] = x[u];
    __syncthreads();
    if (tile + 1 < te) load(tile + 1);
    f32x4 t1[4], t2[4], t3[4];
    mm_tile<kReal>(Xs, kMmK + 1, Ms, kMmK + 1, true, K4, t1, t2, t3);
    const long long l0 = tile * 64;
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const long long r = l0 + 16 * wv + 4 * (l >> 4) + v;
        const int o = o0 + 16 * j + (l & 15);
        if (r < lines && o < nout) out[size_t(r) * nout + o] = mm_result<kReal>(t1[j], t2[j], t3[j], v);
      }
  }
}

typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

// The last interpolation pass (along x, real sinc matrix) with the coil
// normalisation c[:, v] /= ||c[:, v]||_2 fused in: in = [Q][rows][nin], out =
// [Q][rows][nout].  A 64-line tile holds G = 64 / Q row indices times all Q
// coils (local line g Q + q), so every output voxel of the tile has its Q
// coil values in the tile; a zero sum of squares leaves the values as they
// are.
// Products on the FP16 matrix cores with split operands: X and M scaled by
// 2^10 (|X| stays far below the FP16 range: the unit-modulus references
// interpolated by periodic sinc), each split into an FP16 high part and the
// FP16 rounding of the rest, and the three products hi hi, hi lo, lo hi
// accumulated in FP32 on v_mfma_f32_16x16x32_f16 (K = nin padded to 64 with
// zeros); the dropped lo lo term is below 2^-21 of the product.  M is split
// once per workgroup into LDS, a line tile per step on the fly from its FP32
// staging.  Operand lanes of the 16 x 16 x 32 shape: lane l supplies A row
// l % 16 and B column l % 16 for k = 8 (l / 16) + 0..7.
// The sums over q: kQW = Q / 16 waves per row index (Q = 16 or 32) reduce in
// registers and across lanes, and for two waves add the partner wave's
// partial through LDS; any other Q (kQW = 0) puts the squared magnitudes in
// LDS over Xs (free until the next tile is staged) and one thread per
// (g, column) sums them.
template <int kQW>
__global__ void __launch_bounds__(256) k_interp_x_rss(const float2* __restrict__ in,
                                                      float2* __restrict__ out,
                                                      const float2* __restrict__ M, int Qarg,
                                                      long long rows, int nin, int nout) {
  constexpr int XS = 65;  // Xs row stride (float2)
  constexpr int MS = 72;  // Mh, Ml row stride (halves; rows 16-byte aligned)
  __shared__ float2 Xs[64 * XS];
  __shared__ _Float16 Mh[64 * MS], Ml[64 * MS];
  __shared__ float psum[4][64];  // kQW = 2: per-wave column sums
  float* ssq = reinterpret_cast<float*>(Xs);  // kQW = 0: [64 lines][64 columns]
  float* inv = ssq + 64 * 64;                 // kQW = 0: [G][64 columns]
  const int Q = kQW > 0 ? 16 * kQW : Qarg;    // a constant for kQW > 0
  const float scale = 1024.f, unscale = 1.f / (1024.f * 1024.f);
  const int G = 64 / Q;
  const int otiles = (nout + 63) / 64;
  const long long tiles = (rows + G - 1) / G;
  const long long lb = xcd_block(blockIdx.x, gridDim.x);
  const int o0 = int(lb % otiles) * 64;
  const long long tb = lb / otiles * kMmTiles;
  const long long te = tiles < tb + kMmTiles ? tiles : tb + kMmTiles;
  for (int e = threadIdx.x; e < 64 * 64; e += 256) {
    const int o = e >> 6, k = e & 63;
    const float v = (o0 + o < nout && k < nin ? M[size_t(o0 + o) * nin + k].x : 0.f) * scale;
    const _Float16 hi = static_cast<_Float16>(v);
    Mh[o * MS + k] = hi;
    Ml[o * MS + k] = static_cast<_Float16>(v - static_cast<float>(hi));
  }
  // element u of this thread: local line r = e / 64 (= g Q + q), input
  // k = e % 64; its source is line q rows + (tile G + g), at offset off[u] +
  // tile G nin
  int gu[16];
  long long off[16];
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int e = threadIdx.x + 256 * u, r = e >> 6, k = e & 63;
    const int g = r / Q, q = r - g * Q;
    gu[u] = r < G * Q && k < nin ? g : -1;
    off[u] = (1LL * q * rows + g) * nin + k;
  }
  float2 x[16];
  auto load = [&](long long tile) {
    const long long r0 = tile * G;
#pragma unroll
    for (int u = 0; u < 16; ++u)
      x[u] = gu[u] >= 0 && r0 + gu[u] < rows ? in[off[u] + r0 * nin] : make_float2(0.f, 0.f);
  };
  const int l = threadIdx.x & 63, wv = threadIdx.x >> 6, li = l & 15, kg = l >> 4;
  if (tb < te) load(tb);
  for (long long tile = tb; tile < te; ++tile) {
    __syncthreads();  // the previous tile is done with Xs and psum
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = threadIdx.x + 256 * u;
      Xs[(e >> 6) * XS + (e & 63)] = x[u];
    }
    __syncthreads();
    if (tile + 1 < te) load(tile + 1);
    f32x4 t1[4], t2[4];  // Re and Im: rows 4 kg + v of the wave's 16 lines
#pragma unroll
    for (int j = 0; j < 4; ++j) t1[j] = t2[j] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
      const int k0 = 32 * ks + 8 * kg;
      f16x8 rh, rl, ih, il;
      const float2* xr = Xs + (16 * wv + li) * XS + k0;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const float2 v = xr[i];
        const float a = v.x * scale, b = v.y * scale;
        const _Float16 ah = static_cast<_Float16>(a), bh = static_cast<_Float16>(b);
        rh[i] = ah;
        rl[i] = static_cast<_Float16>(a - static_cast<float>(ah));
        ih[i] = bh;
        il[i] = static_cast<_Float16>(b - static_cast<float>(bh));
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int o = 16 * j + li;
        const f16x8 mh = *reinterpret_cast<const f16x8*>(Mh + o * MS + k0);
        const f16x8 ml = *reinterpret_cast<const f16x8*>(Ml + o * MS + k0);
        t1[j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(rh, mh, t1[j], 0, 0, 0);
        t1[j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(rh, ml, t1[j], 0, 0, 0);
        t1[j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(rl, mh, t1[j], 0, 0, 0);
        t2[j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ih, mh, t2[j], 0, 0, 0);
        t2[j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ih, ml, t2[j], 0, 0, 0);
        t2[j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(il, mh, t2[j], 0, 0, 0);
      }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      t1[j] = t1[j] * unscale;
      t2[j] = t2[j] * unscale;
    }
    float sc[4];  // 1 / norm for the lane's columns 16 j + l % 16
    if (kQW > 0) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        float s = 0.f;
#pragma unroll
        for (int v = 0; v < 4; ++v) s += t1[j][v] * t1[j][v] + t2[j][v] * t2[j][v];
        s += __shfl_xor(s, 16, 64);
        s += __shfl_xor(s, 32, 64);
        sc[j] = s;
      }
      if (kQW == 2) {
        if (l < 16)
#pragma unroll
          for (int j = 0; j < 4; ++j) psum[wv][16 * j + l] = sc[j];
        __syncthreads();
#pragma unroll
        for (int j = 0; j < 4; ++j) sc[j] += psum[wv ^ 1][16 * j + li];
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) sc[j] = sc[j] > 0.f ? 1.f / sqrtf(sc[j]) : 1.f;
    } else {
      __syncthreads();  // every wave is done reading Xs
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          ssq[(16 * wv + 4 * kg + v) * 64 + 16 * j + li] =
              t1[j][v] * t1[j][v] + t2[j][v] * t2[j][v];
      __syncthreads();
      for (int e = threadIdx.x; e < G * 64; e += 256) {
        const int g = e >> 6, c = e & 63;
        float s = 0.f;
        for (int q = 0; q < Q; ++q) s += ssq[(g * Q + q) * 64 + c];
        inv[e] = s > 0.f ? 1.f / sqrtf(s) : 1.f;
      }
      __syncthreads();
    }
    const long long r0 = tile * G;
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = 16 * wv + 4 * kg + v, c = 16 * j + li;
        const int g = r / Q, q = r - g * Q;
        if (r < G * Q && r0 + g < rows && o0 + c < nout)
          out[(size_t(q) * rows + r0 + g) * nout + o0 + c] =
              cscale(make_float2(t1[j][v], t2[j][v]), kQW > 0 ? sc[j] : inv[g * 64 + c]);
      }
  }
}

pisco_status_t interp_x_rss(Handle* h, const float2* in, float2* out, const float2* M, int Q,
                            long long rows, int nin, int nout) {
  if (Q < 1 || Q > 64 || nin < 1 || nin > kMmK || nout < 1 || rows < 1)
    return PISCO_ERR_UNSUPPORTED;
  const long long tiles = (rows + 64 / Q - 1) / (64 / Q);
  const long long blocks = 1LL * ceil_div(nout, 64) * ceil_div(tiles, kMmTiles);
  if (blocks >= (1LL << 24)) return PISCO_ERR_UNSUPPORTED;
  if (Q == 16)
    PISCO_KERNEL(h, k_interp_x_rss<1>, dim3(unsigned(blocks)), dim3(256), 0, in, out, M, Q, rows,
                 nin, nout);
  else if (Q == 32)
    PISCO_KERNEL(h, k_interp_x_rss<2>, dim3(unsigned(blocks)), dim3(256), 0, in, out, M, Q, rows,
                 nin, nout);
  else
    PISCO_KERNEL(h, k_interp_x_rss<0>, dim3(unsigned(blocks)), dim3(256), 0, in, out, M, Q, rows,
                 nin, nout);
  return PISCO_OK;
}

template <class TI, class TO>
static pisco_status_t axis_impl(Handle* h, const TI* in, TO* out, const int shape_in[4],
                                int axis, int nout, const TO* M, bool real_m, int epi = 0,
                                int epi_q = 0, float epi_bound = 0.f) {
  long long outer = shape_in[0];
  for (int d = 1; d < axis; ++d) outer *= shape_in[d];
  long long inner = 1;
  for (int d = axis + 1; d < 4; ++d) inner *= shape_in[d];
  const int nin = shape_in[axis];
  // the matrix-core kernels: FP32, at most kMmK inputs, enough work to fill
  // the chip, and column tiles at least half used
  const long long mm_blocks =
      ceil_div(nout, 64) * ceil_div(inner == 1 ? ceil_div(outer, 64) : outer * ceil_div(inner, 64),
                                    kMmTiles);
  if (sizeof(TI) == sizeof(float2) && sizeof(TO) == sizeof(float2) && nin <= kMmK &&
      outer * inner * nout >= (1LL << 22) && (inner == 1 || inner >= 32) &&
      mm_blocks < (1LL << 24)) {
    const float2* fi = reinterpret_cast<const float2*>(in);
    float2* fo = reinterpret_cast<float2*>(out);
    const float2* fm = reinterpret_cast<const float2*>(M);
    if (inner == 1) {
      if (epi != 0) return PISCO_ERR_UNSUPPORTED;
      if (real_m)
        PISCO_KERNEL(h, k_axis_mm_lines<true>, dim3(unsigned(mm_blocks)), dim3(256), 0, fi, fo,
                     fm, outer, nin, nout);
      else
        PISCO_KERNEL(h, k_axis_mm_lines<false>, dim3(unsigned(mm_blocks)), dim3(256), 0, fi, fo,
                     fm, outer, nin, nout);
    } else {
      if (epi == 1 && !real_m)
        PISCO_KERNEL(h, (k_axis_mm_cols<false, 1>), dim3(unsigned(mm_blocks)), dim3(256), 0, fi,
                     fo, fm, outer, nin, nout, int(inner), epi_q, epi_bound);
      else if (epi != 0)
        return PISCO_ERR_UNSUPPORTED;
      else if (real_m)
        PISCO_KERNEL(h, (k_axis_mm_cols<true, 0>), dim3(unsigned(mm_blocks)), dim3(256), 0, fi,
                     fo, fm, outer, nin, nout, int(inner), 0, 0.f);
      else
        PISCO_KERNEL(h, (k_axis_mm_cols<false, 0>), dim3(unsigned(mm_blocks)), dim3(256), 0, fi,
                     fo, fm, outer, nin, nout, int(inner), 0, 0.f);
    }
    return PISCO_OK;
  }
  if (epi != 0) return PISCO_ERR_UNSUPPORTED;
  if (inner == 1) {
    int lpb = nout >= 256 ? 1 : 256 / nout;
    const int fit = int((64 * 1024) / (size_t(nin) * sizeof(TO)));  // staged lines in 64 KB
    lpb = lpb < fit ? lpb : fit;
    const int per = (nout + 255) / 256;
    const size_t lds = size_t(lpb) * nin * sizeof(TO);
    if (lpb < 1) return PISCO_ERR_UNSUPPORTED;
    const long long blocks = per > 1 ? outer * per : ceil_div(outer, lpb);
    PISCO_KERNEL(h, (k_axis_last<TI, TO>), dim3(blocks), dim3(256), lds, in, out, M, outer, nin,
                 nout, lpb);
  } else if (sizeof(TO) == sizeof(double2) && nin <= 32 && outer * inner >= 256LL * 1024) {
    // short FP64 transforms over long runs (the structured Gram products)
    const long long cols = ceil_div(outer * inner, 256);
    const double2* Md = reinterpret_cast<const double2*>(M);
    double2* od = reinterpret_cast<double2*>(out);
    if (nin <= 16)
      PISCO_KERNEL(h, (k_axis_reg<TI, 16>), dim3(cols), dim3(256), 0, in, od, Md, outer, nin,
                   nout, int(inner));
    else
      PISCO_KERNEL(h, (k_axis_reg<TI, 32>), dim3(cols), dim3(256), 0, in, od, Md, outer, nin,
                   nout, int(inner));
  } else {
    if (nin > kMidMaxIn) return PISCO_ERR_UNSUPPORTED;
    const long long cols = ceil_div(outer * inner, 256);
    if (cols * ceil_div(nout, 16) >= 1024)
      PISCO_KERNEL(h, (k_axis_mid<TI, TO, 16>), dim3(cols, ceil_div(nout, 16)), dim3(256), 0, in,
                   out, M, outer, nin, nout, int(inner));
    else
      PISCO_KERNEL(h, (k_axis_mid<TI, TO, 4>), dim3(cols, ceil_div(nout, 4)), dim3(256), 0, in,
                   out, M, outer, nin, nout, int(inner));
  }
  return PISCO_OK;
}

pisco_status_t axis_transform(Handle* h, const float2* in, float2* out, const int shape_in[4],
                              int axis, int nout, const float2* M, bool real_m) {
  return axis_impl<float2, float2>(h, in, out, shape_in, axis, nout, M, real_m);
}

pisco_status_t axis_transform_gx(Handle* h, const float2* in, float2* out,
                                 const int shape_in[4], int axis, int nout, const float2* M,
                                 int Q, float bound) {
  long long outer = shape_in[0];
  for (int d = 1; d < axis; ++d) outer *= shape_in[d];
  if (Q < 1 || outer != 1LL * Q * (Q + 1) / 2) return PISCO_ERR_UNSUPPORTED;
  return axis_impl<float2, float2>(h, in, out, shape_in, axis, nout, M, false, 1, Q, bound);
}

pisco_status_t axis_transform64(Handle* h, const float2* in, double2* out,
                                const int shape_in[4], int axis, int nout, const double2* M) {
  return axis_impl<float2, double2>(h, in, out, shape_in, axis, nout, M, false);
}

pisco_status_t axis_transform64(Handle* h, const double2* in, double2* out,
                                const int shape_in[4], int axis, int nout, const double2* M) {
  return axis_impl<double2, double2>(h, in, out, shape_in, axis, nout, M, false);
}

// ------------------------------------------------------------------ plan-constant tables

// One kernel builds every table a call needs: blockIdx.y selects the job,
// the blocks of a row stride over its elements.
//   dft  : M[o][i] = scale * w(i) * exp(i sign 2 pi (i - ci)(o - co) / period),
//          w(i) = exp(-(i - ci)^2 / (2 sigma^2)) when sigma > 0, else 1
//          (float2 or double2 entries)
//   sinc : periodic sinc (Dirichlet) interpolation from nin to nout >= nin
//          (float2 or double2 entries)
//          centred samples, M[o][a] = (1/nin) sum_k w_k exp(i 2 pi k (y_o - x_a))
//          over the centred band of nin frequencies, the -nin/2 term split
//          in half onto +-nin/2 when nin is even and nout > nin
//   support : the points n of the box with ||n||_2 <= radius (or the whole
//          box for the rectangular support), lexicographic (z slowest), as
//          int4 (z, y, x, 0)
//   boxmap : box cell -> index of its point in the support list, -1 outside;
//          the index of an inside cell is the number of inside cells before
//          it in the same lexicographic order
enum TableKind { kTDft32 = 0, kTDft64 = 1, kTSinc32 = 2, kTSupport = 3, kTBoxMap = 4,
                 kTSinc64 = 5, kTDftDft32 = 6 };
constexpr int kMaxTableJobs = 24;
struct TableJob {
  int kind, nout, nin, co, ci;
  double period, sign, scale, sigma;
  void* out;
  // kTDftDft32: the product of two dft matrices, [nout][nmid] (the fields
  // above, no weight) times [nmid][nin] (these), summed over the middle index
  int nmid, co2, ci2;
  double period2, sign2, scale2;
};
struct TableJobs {
  TableJob job[kMaxTableJobs];
  int count;
  int D, tau, tz;  // support box: x, y in [-tau, tau], z in [-tz, tz]
  double r2;       // radius^2 (ellipsoid); a negative value: the whole box
};

__device__ inline bool in_ball(int z, int y, int x, double r2) {
  return r2 < 0.0 || double(z) * z + double(y) * y + double(x) * x <= r2;
}

__device__ void dft_value(int o, int i, int co, int ci, double period, double sign,
                          double scale, double sigma, double* re, double* im) {
  const long long prod = 1LL * (i - ci) * (o - co);
  // the phase reduced exactly in integers before the trigonometric call
  const long long per = (long long)llround(period);
  double frac;
  if (double(per) == period && per > 0) {
    long long r = prod % per;
    if (r < 0) r += per;
    frac = double(r) / period;
  } else {
    frac = double(prod) / period;
  }
  double sn, cs;
  sincospi(2.0 * sign * frac, &sn, &cs);
  double w = scale;
  if (sigma > 0.0) {
    const double k = double(i - ci);
    w *= exp(-k * k / (2.0 * sigma * sigma));
  }
  *re = w * cs;
  *im = w * sn;
}

__device__ void dft_entry(const TableJob& j, int idx, double* re, double* im) {
  const int o = idx / j.nin, i = idx - o * j.nin;
  dft_value(o, i, j.co, j.ci, j.period, j.sign, j.scale, j.sigma, re, im);
}

// entry (o, i) of the product of the two dft matrices of a kTDftDft32 job
__device__ void dftdft_entry(const TableJob& j, int idx, double* re, double* im) {
  const int o = idx / j.nin, i = idx - o * j.nin;
  double sr = 0.0, si = 0.0;
  for (int m = 0; m < j.nmid; ++m) {
    double ar, ai, br, bi;
    dft_value(o, m, j.co, j.ci, j.period, j.sign, j.scale, 0.0, &ar, &ai);
    dft_value(m, i, j.co2, j.ci2, j.period2, j.sign2, j.scale2, 0.0, &br, &bi);
    sr += ar * br - ai * bi;
    si += ar * bi + ai * br;
  }
  *re = sr;
  *im = si;
}

__device__ void sinc_entry(const TableJob& j, int idx, double* re, double* im) {
  const int nout = j.nout, nin = j.nin;
  const int o = idx / nin, a = idx - o * nin;
  const int kmin = -(nin / 2), kmax = (nin + 1) / 2 - 1;
  const bool split = (nin % 2 == 0) && nout > nin;
  const double y = double(o - nout / 2) / double(nout);
  const double x = double(a - nin / 2) / double(nin);
  // The frequencies run over a symmetric range (odd nin, or even nin with the
  // Nyquist term split in halves at -nin/2 and +nin/2), so the sine terms
  // cancel in pairs; for even nin with nout = nin the grids coincide and the
  // sum is nin times a Kronecker delta.  The kernel is real: only the cosine
  // sum is formed, and the interpolation passes take the real-matrix products.
  double sr = 0.0;
  for (int k = kmin; k <= kmax; ++k) {
    const double w = (split && k == kmin) ? 0.5 : 1.0;
    sr += w * cospi(2.0 * double(k) * (y - x));
  }
  if (split) sr += 0.5 * cospi(2.0 * double(nin / 2) * (y - x));
  *re = sr / nin;
  *im = 0.0;
}

__global__ void __launch_bounds__(256) k_build_tables(TableJobs jobs) {
  const TableJob& j = jobs.job[blockIdx.y];
  const int box = 2 * jobs.tau + 1, bz = 2 * jobs.tz + 1;
  const int ncell = bz * box * box;
  int total = 0;
  switch (j.kind) {
    case kTSupport: total = 1; break;
    case kTBoxMap: total = ncell; break;
    default: total = j.nout * j.nin;
  }
  for (int idx = blockIdx.x * 256 + threadIdx.x; idx < total; idx += gridDim.x * 256) {
    if (j.kind == kTDft32 || j.kind == kTDft64 || j.kind == kTSinc32 || j.kind == kTSinc64 ||
        j.kind == kTDftDft32) {
      double re, im;
      if (j.kind == kTSinc32 || j.kind == kTSinc64)
        sinc_entry(j, idx, &re, &im);
      else if (j.kind == kTDftDft32)
        dftdft_entry(j, idx, &re, &im);
      else
        dft_entry(j, idx, &re, &im);
      if (j.kind == kTDft64 || j.kind == kTSinc64)
        static_cast<double2*>(j.out)[idx] = make_double2(re, im);
      else
        static_cast<float2*>(j.out)[idx] = make_float2(float(re), float(im));
    } else if (j.kind == kTSupport) {
      // sequential enumeration (one thread): the order is the definition
      int c = 0;
      int4* out = static_cast<int4*>(j.out);
      for (int z = -jobs.tz; z <= jobs.tz; ++z)
        for (int y = -jobs.tau; y <= jobs.tau; ++y)
          for (int x = -jobs.tau; x <= jobs.tau; ++x)
            if (in_ball(z, y, x, jobs.r2)) out[c++] = make_int4(z, y, x, 0);
    } else {
      const int cz = idx / (box * box), rem = idx - cz * box * box;
      const int cy = rem / box, cx = rem - cy * box;
      int v = -1;
      if (in_ball(cz - jobs.tz, cy - jobs.tau, cx - jobs.tau, jobs.r2)) {
        v = 0;
        for (int e = 0; e < idx; ++e) {
          const int ez = e / (box * box), er = e - ez * box * box;
          const int ey = er / box, ex = er - ey * box;
          v += in_ball(ez - jobs.tz, ey - jobs.tau, ex - jobs.tau, jobs.r2) ? 1 : 0;
        }
      }
      static_cast<int*>(j.out)[idx] = v;
    }
  }
}

size_t layout_tables(const Plan& p, unsigned which, void* ws, Tables* out) {
  Carver c(ws);
  Tables t;
  const int first = p.D == 3 ? 0 : 1;
  const int box = 2 * p.tau + 1;
  if (which & (kTabSupport | kTabGx | kTabToeplitz)) t.sup = c.take<int4>(p.L);
  if (which & (kTabGx | kTabToeplitz))
    t.boxmap = c.take<int>(size_t(p.D == 3 ? box : 1) * box * box);
  if (which & kTabToeplitz) {
    const int F = p.K[2];
    t.Tf = c.take<double2>(size_t(F) * box);
    t.Ti = c.take<double2>(size_t(box) * F);
    t.Tr = c.take<double2>(size_t(F) * F);
  }
  if (which & kTabGx) {
    for (int d = first; d < 3; ++d) {
      t.M1[d] = c.take<float2>(size_t(p.K[d]) * box);
      t.M4[d] = c.take<float2>(size_t(p.lr[d]) * p.K[d]);
    }
  }
  if (which & kTabMaps) {
    for (int d = first; d < 3; ++d) {
      t.Ma[d] = c.take<double2>(size_t(p.lr[d]) * p.acs[d]);
      t.Ms[d] = c.take<float2>(size_t(p.out[d]) * p.lr[d]);
    }
  }
  if (which & kTabMask)
    for (int d = first; d < 3; ++d) t.Ms64[d] = c.take<double2>(size_t(p.out[d]) * p.lr[d]);
  if (out) *out = t;
  return c.used + 256;
}

pisco_status_t build_tables(Handle* h, const Plan& p, unsigned which, const Tables& t) {
  TableJobs jobs{};
  jobs.D = p.D;
  jobs.tau = p.tau;
  jobs.tz = p.D == 3 ? p.tau : 0;
  jobs.r2 = p.shape == PISCO_SHAPE_RECTANGLE ? -1.0 : double(p.radius) * double(p.radius);
  int maxel = 1;
  auto add = [&](int kind, void* out, int nout, int nin, int co, int ci, double period,
                 double sign, double scale, double sigma) {
    TableJob& j = jobs.job[jobs.count++];
    j.kind = kind;
    j.out = out;
    j.nout = nout;
    j.nin = nin;
    j.co = co;
    j.ci = ci;
    j.period = period;
    j.sign = sign;
    j.scale = scale;
    j.sigma = sigma;
    const int n = kind == kTSupport ? 1 : nout * nin;
    maxel = n > maxel ? n : maxel;
  };
  const int first = p.D == 3 ? 0 : 1;
  const int tau = p.tau, box = 2 * tau + 1;
  if (t.sup && (which & (kTabSupport | kTabGx | kTabToeplitz)))
    add(kTSupport, t.sup, 1, 1, 0, 0, 1, 0, 0, 0);
  if (which & (kTabGx | kTabToeplitz))
    add(kTBoxMap, t.boxmap, (p.D == 3 ? box : 1) * box, box, 0, 0, 1, 0, 0, 0);
  if (which & kTabToeplitz) {
    // structured Gram products on F = 4 tau + 1 points per axis: box (m -
    // tau) -> frequency e^{-i 2 pi f m / F}; back with e^{+i 2 pi f n / F} / F;
    // lags (d - 2 tau) -> frequency e^{-i 2 pi f d / F}
    const int F = p.K[2];
    add(kTDft64, t.Tf, F, box, 0, tau, F, -1.0, 1.0, 0.0);
    add(kTDft64, t.Ti, box, F, tau, 0, F, +1.0, 1.0 / F, 0.0);
    add(kTDft64, t.Tr, F, F, 0, 2 * tau, F, -1.0, 1.0, 0.0);
  }
  if (which & kTabGx) {
    for (int d = first; d < 3; ++d) {
      const int Lk = p.K[d], Bd = p.B[d], lr = p.lr[d];
      // filter spectra: e^{+i 2 pi n f / Lk}, n = box index - tau
      add(kTDft32, t.M1[d], Lk, box, 0, tau, Lk, +1.0, 1.0, 0.0);
      // low-res evaluation straight from the spectra: the lags (1/Lk) e^{+i 2
      // pi m f / Lk}, m = lag index - 2 tau, evaluated at e^{-i 2 pi m x}, x =
      // (a - floor(N/2)) / N, summed over the Bd lags in FP64
      add(kTDft32, t.M4[d], lr, Lk, lr / 2, 2 * tau, lr, -1.0, 1.0, 0.0);
      TableJob& j = jobs.job[jobs.count - 1];
      j.kind = kTDftDft32;
      j.nmid = Bd;
      j.co2 = 2 * tau;
      j.ci2 = 0;
      j.period2 = Lk;
      j.sign2 = +1.0;
      j.scale2 = 1.0 / Lk;
    }
  }
  if (which & kTabMaps) {
    for (int d = first; d < 3; ++d) {
      const int A = p.acs[d], n = p.lr[d];
      // apodized reconstruction on the low-res grid, Gaussian of width A/4
      add(kTDft64, t.Ma[d], n, A, n / 2, A / 2, n, +1.0, 1.0, A / 4.0);
      add(kTSinc32, t.Ms[d], p.out[d], n, 0, 0, 1, 0, 0, 0);
    }
  }
  if (which & kTabMask)
    for (int d = first; d < 3; ++d) add(kTSinc64, t.Ms64[d], p.out[d], p.lr[d], 0, 0, 1, 0, 0, 0);
  if (jobs.count == 0) return PISCO_OK;
  const unsigned gx = ceil_div(maxel, 256) < 64 ? ceil_div(maxel, 256) : 64;
  PISCO_KERNEL(h, k_build_tables, dim3(gx, jobs.count), dim3(256), 0, jobs);
  return PISCO_OK;
}

}  // namespace pisco
