// Learned warm start for the per-voxel power iteration (not in the paper;
// the iteration it feeds is Sec. IV-E's).
//
// A small network maps each voxel's G(x) and a neighbour eigenvector to a
// start vector close to the eigenvector of G(x) for its smallest eigenvalue:
//   z = [G_qq / |Lambda| (Q), Re/Im G_pq / |Lambda| for p < q (Q(Q-1)),
//        Re/Im n (2Q)]
//   h1 = relu(W1 z + b1), h2 = relu(W2 h1 + b2), y = W3 h2 + b3 (2Q reals)
//   c_hat = n + y  (complex; a correction of the neighbour vector n)
// n is the eigenvector at the parent voxel of a grid coarser by two per
// dimension (solved first from the plain start), its largest entry rotated
// real and positive.  Training minimises the gauge-invariant loss
// 1 - |c_hat^H c|^2 / ||c_hat||^2 against the method's own eigenvectors c,
// with Adam on FP32 master weights.
//
// Arithmetic: weights FP16, products on the matrix cores
// (v_mfma_f32_16x16x32_f16) with FP32 accumulation.  Inference carries the
// activations in FP16.  Training carries features, activations and
// per-voxel gradients as FP16 pairs hi + lo (FP32 values; products hi hi +
// hi lo + lo hi), because with one FP16 part the rounding of an activation
// moves pre-activations near zero across the ReLU and the flipped masks
// dominate the gradient error (about 1e-2 in the 2-norm); the weight
// gradients are summed over the voxels by split K in FP32, then the loss,
// gradients and optimizer state are FP32.
//
// Parameter vector (FP32 master and FP16 copy, same layout):
//   [W1 (H x Din, row-major), b1 (H), W2 (H x H), b2 (H), W3 (Dout x H), b3]
// with Din = Q^2 + 2Q, H = 256, Dout = 2Q.
#include <cfloat>
#include <cmath>

#include "common.hpp"

namespace pisco {

namespace {

constexpr int kHidden = 256;

typedef float f32x4 __attribute__((ext_vector_type(4)));

struct WsDims {
  int Q, din, h, dout;
  long long off_w1, off_b1, off_w2, off_b2, off_w3, off_b3, count;
};

WsDims ws_dims(int Q) {
  WsDims d;
  d.Q = Q;
  d.din = Q * Q + 2 * Q;
  d.h = kHidden;
  d.dout = 2 * Q;
  d.off_w1 = 0;
  d.off_b1 = d.off_w1 + 1LL * d.h * d.din;
  d.off_w2 = d.off_b1 + d.h;
  d.off_b2 = d.off_w2 + 1LL * d.h * d.h;
  d.off_w3 = d.off_b2 + d.h;
  d.off_b3 = d.off_w3 + 1LL * d.dout * d.h;
  d.count = d.off_b3 + d.dout;
  return d;
}

__device__ inline int pair_index(int p, int q, int Q) {  // p <= q
  return p * Q - p * (p - 1) / 2 + (q - p);
}

// ------------------------------------------------------------------ features

// X[j][v] (feature-major Din x N, FP16; with Xlo the FP32 value as hi +
// lo) from packed G ([pair][N] float2) and the neighbour vectors ([Q][N]
// float2), one thread per voxel: every read and write is contiguous across
// the voxels of a wave (the loops over the kMaxQ bound are unrolled and
// guarded by Q).
__global__ void __launch_bounds__(256) k_ws_features(const float2* __restrict__ G,
                                                     const float2* __restrict__ nb, int Q,
                                                     long long N, float inv_bound,
                                                     _Float16* __restrict__ X,
                                                     _Float16* __restrict__ Xlo) {
  const long long v = blockIdx.x * 256LL + threadIdx.x;
  if (v >= N) return;
  auto put = [&](int j, float f) {
    const _Float16 hi = static_cast<_Float16>(f);
    X[size_t(j) * N + v] = hi;
    if (Xlo) Xlo[size_t(j) * N + v] = static_cast<_Float16>(f - static_cast<float>(hi));
  };
  // diagonal (real), then the off-diagonal entries p < q in row-major order
  // (re, im)
  int k = 0, o = 0;
#pragma unroll
  for (int p = 0; p < kMaxQ; ++p) {
#pragma unroll
    for (int q = p; q < kMaxQ; ++q) {
      if (p < Q && q < Q) {
        const float2 g = G[size_t(k) * N + v];
        ++k;
        if (p == q) {
          put(p, g.x * inv_bound);
        } else {
          put(Q + 2 * o, g.x * inv_bound);
          put(Q + 2 * o + 1, g.y * inv_bound);
          ++o;
        }
      }
    }
  }
#pragma unroll
  for (int q = 0; q < kMaxQ; ++q) {
    if (q >= Q) continue;
    const float2 n = nb[size_t(q) * N + v];
    put(Q * Q + 2 * q, n.x);
    put(Q * Q + 2 * q + 1, n.y);
  }
}

// ------------------------------------------------------------------ GEMM

// C (M x N) = sum over operand parts of op(A_a) op(B_b), FP16 operands with
// FP32 accumulation on the matrix cores (v_mfma_f32_16x16x32_f16).  An
// operand is one FP16 matrix or a pair hi + lo of the same layout (an FP32
// value carried as two FP16 parts); with pairs the products hi hi, hi lo
// and lo hi are summed (lo lo, below 2^-22 relative, is dropped).
// op(A)(m, k) = kTA ? A[k lda + m] : A[m lda + k];
// op(B)(k, n) = kTB ? B[n ldb + k] : B[k ldb + n].
// Workgroup tile 64 x 64, four waves of 32 x 32 (2 x 2 blocks of 16 x 16),
// K in steps of 32 through LDS: each operand tile is staged as 64 rows of
// 32 k (row stride 40 halves, so that the 16-byte operand reads of eight
// lanes hit distinct banks), double-buffered, the next step's global loads
// in flight during the current step's products.  A k-contiguous operand is
// loaded eight halves per thread along k; an m-contiguous one eight along m
// and transposed on its way into LDS.  Operand lanes: lane l supplies row l
// % 16 at k = 8 (l / 16) + j (both operands the same, so any assignment of
// k to the lanes gives the same sums); accumulator element v of lane l is
// row 4 (l / 16) + v, column l % 16.  blockIdx.z takes K chunk z of kchunk
// (split K: the partial products go to C + z M N, summed by k_ws_reduce).
// Epilogues:
enum : int {
  kEpiBiasReluF16 = 0,    // C16 = fp16(max(acc + bias[n], 0))
  kEpiBiasReluSplit = 1,  // (C16, C16lo) = hi / lo parts of max(acc + bias[n], 0)
  kEpiBiasF32 = 2,        // C32 = acc + bias[n]
  kEpiMaskSplit = 3,      // (C16, C16lo) = parts of acc where the mask pair is > 0, else 0
  kEpiPartF32 = 4,        // C32 + z M N = acc (ldc = N)
};

typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

constexpr int kGT = 64;        // tile rows (M) and columns (N)
constexpr int kGK = 32;        // K step
constexpr int kGS = kGK + 8;   // LDS row stride, halves

struct HOperand {
  const _Float16* part[2];  // hi, lo (lo null for a single FP16 operand)
  int ld;
  bool vec;  // ld and both parts allow 16-byte loads
};

struct HOut {
  void* c;             // FP16 (hi) or FP32 output
  _Float16* clo;       // lo part for split epilogues
  int ldc;
  const _Float16* bias;
  const _Float16* mask[2];  // mask pair (hi, lo): on where hi > 0 or lo > 0
  int ldm;
};

// eight halves of op(X) for this thread's share of the tile (rows r0.., k0..)
template <bool kKc>
__device__ inline f16x8 tile_load(const _Float16* base, int ld, bool vec, int R, int K, int r0,
                                  int k0) {
  const int t = threadIdx.x;
  f16x8 v;
  if (kKc) {  // element (r, k) at base[r ld + k]
    const int r = r0 + (t >> 2), k = k0 + (t & 3) * 8;
    if (vec && r < R && k + 8 <= K) return *reinterpret_cast<const f16x8*>(base + size_t(r) * ld + k);
#pragma unroll
    for (int i = 0; i < 8; ++i)
      v[i] = r < R && k + i < K ? base[size_t(r) * ld + k + i] : static_cast<_Float16>(0.f);
  } else {  // element (r, k) at base[k ld + r]
    const int k = k0 + (t >> 3), r = r0 + (t & 7) * 8;
    if (vec && k < K && r + 8 <= R) return *reinterpret_cast<const f16x8*>(base + size_t(k) * ld + r);
#pragma unroll
    for (int i = 0; i < 8; ++i)
      v[i] = k < K && r + i < R ? base[size_t(k) * ld + r + i] : static_cast<_Float16>(0.f);
  }
  return v;
}

template <bool kKc>
__device__ inline void tile_store(_Float16* lds, const f16x8& v) {
  const int t = threadIdx.x;
  if (kKc) {
    *reinterpret_cast<f16x8*>(lds + (t >> 2) * kGS + (t & 3) * 8) = v;
  } else {
    const int k = t >> 3, r = (t & 7) * 8;
#pragma unroll
    for (int i = 0; i < 8; ++i) lds[(r + i) * kGS + k] = v[i];
  }
}

template <bool kTA, bool kTB, int kPA, int kPB, int kEpi>
__global__ void __launch_bounds__(256) k_hgemm(HOperand A, HOperand B, int M, int N, int K,
                                               int kchunk, HOut o) {
  __shared__ _Float16 As[2][kPA][kGT * kGS];
  __shared__ _Float16 Bs[2][kPB][kGT * kGS];
  const int t = threadIdx.x, wv = t >> 6, l = t & 63;
  const int li = l & 15, kg = l >> 4;
  const int m0 = blockIdx.x * kGT, n0 = blockIdx.y * kGT;
  const int wm = (wv & 1) * 32, wn = (wv >> 1) * 32;
  const int kb = blockIdx.z * kchunk, ke = K < kb + kchunk ? K : kb + kchunk;
  f32x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  f16x8 ra[kPA], rb[kPB];
  auto load = [&](int k0) {
#pragma unroll
    for (int p = 0; p < kPA; ++p) ra[p] = tile_load<!kTA>(A.part[p], A.ld, A.vec, M, ke, m0, k0);
#pragma unroll
    for (int p = 0; p < kPB; ++p) rb[p] = tile_load<kTB>(B.part[p], B.ld, B.vec, N, ke, n0, k0);
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int p = 0; p < kPA; ++p) tile_store<!kTA>(As[buf][p], ra[p]);
#pragma unroll
    for (int p = 0; p < kPB; ++p) tile_store<kTB>(Bs[buf][p], rb[p]);
  };
  int buf = 0;
  if (kb < ke) {
    load(kb);
    store(0);
  }
  __syncthreads();
  for (int k0 = kb; k0 < ke; k0 += kGK) {
    const bool next = k0 + kGK < ke;
    if (next) load(k0 + kGK);
    f16x8 a[kPA][2], b[kPB][2];
#pragma unroll
    for (int p = 0; p < kPA; ++p)
#pragma unroll
      for (int i = 0; i < 2; ++i)
        a[p][i] = *reinterpret_cast<const f16x8*>(&As[buf][p][(wm + 16 * i + li) * kGS + 8 * kg]);
#pragma unroll
    for (int p = 0; p < kPB; ++p)
#pragma unroll
      for (int j = 0; j < 2; ++j)
        b[p][j] = *reinterpret_cast<const f16x8*>(&Bs[buf][p][(wn + 16 * j + li) * kGS + 8 * kg]);
#pragma unroll
    for (int pa = 0; pa < kPA; ++pa)
#pragma unroll
      for (int pb = 0; pb < kPB; ++pb) {
        if (pa + pb > 1) continue;  // lo lo dropped
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a[pa][i], b[pb][j], acc[i][j], 0,
                                                               0, 0);
      }
    if (next) store(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int m = m0 + wm + 16 * i + 4 * kg + v, n = n0 + wn + 16 * j + li;
        if (m >= M || n >= N) continue;
        float x = acc[i][j][v];
        if (kEpi == kEpiPartF32) {
          static_cast<float*>(o.c)[(size_t(blockIdx.z) * M + m) * N + n] = x;
          continue;
        }
        if (kEpi == kEpiBiasF32) {
          static_cast<float*>(o.c)[size_t(m) * o.ldc + n] = x + static_cast<float>(o.bias[n]);
          continue;
        }
        if (kEpi == kEpiBiasReluF16 || kEpi == kEpiBiasReluSplit)
          x = fmaxf(x + static_cast<float>(o.bias[n]), 0.f);
        if (kEpi == kEpiMaskSplit) {
          const size_t mi = size_t(m) * o.ldm + n;
          const bool on = static_cast<float>(o.mask[0][mi]) > 0.f ||
                          static_cast<float>(o.mask[1][mi]) > 0.f;
          x = on ? x : 0.f;
        }
        const _Float16 hi = static_cast<_Float16>(x);
        static_cast<_Float16*>(o.c)[size_t(m) * o.ldc + n] = hi;
        if (kEpi != kEpiBiasReluF16)
          o.clo[size_t(m) * o.ldc + n] = static_cast<_Float16>(x - static_cast<float>(hi));
      }
}

// out[i] (+)= sum_z part[z][i], i < n (fixed order)
__global__ void k_ws_reduce(const float* __restrict__ part, int nsplit, long long n,
                            float* __restrict__ out) {
  const long long i = blockIdx.x * 256LL + threadIdx.x;
  if (i >= n) return;
  float s = 0.f;
  for (int z = 0; z < nsplit; ++z) s += part[size_t(z) * n + i];
  out[i] = s;
}

HOperand hop(const _Float16* hi, const _Float16* lo, int ld) {
  HOperand a;
  a.part[0] = hi;
  a.part[1] = lo;
  a.ld = ld;
  auto al = [](const void* p) { return !p || (reinterpret_cast<uintptr_t>(p) & 15) == 0; };
  a.vec = ld % 8 == 0 && al(hi) && al(lo);
  return a;
}

// Largest partial buffer of the split-K weight gradients, floats.
constexpr long long kPartFloats = 1LL << 22;

template <bool kTA, bool kTB, int kPA, int kPB, int kEpi>
pisco_status_t hgemm(Handle* h, const HOperand& A, const HOperand& B, int M, int N, int K,
                     const HOut& o, float* part = nullptr) {
  if (M <= 0 || N <= 0) return PISCO_OK;
  const int mt = ceil_div(M, kGT), nt = ceil_div(N, kGT);
  int nsplit = 1, kchunk = K;
  if (kEpi == kEpiPartF32) {
    // enough workgroups to fill the chip, chunks of whole K steps, the
    // partials within the buffer
    long long want = ceil_div(2048, mt * nt);
    const long long cap = kPartFloats / (1LL * M * N);
    if (want > cap) want = cap;
    if (want < 1) want = 1;
    kchunk = int(ceil_div(ceil_div(K, int(want)), kGK) * kGK);
    if (kchunk < kGK) kchunk = kGK;
    nsplit = ceil_div(K, kchunk);
    if (nsplit < 1) nsplit = 1;
  }
  HOut oo = o;
  if (kEpi == kEpiPartF32) oo.c = part;
  PISCO_KERNEL(h, (k_hgemm<kTA, kTB, kPA, kPB, kEpi>), dim3(mt, nt, nsplit), dim3(256), 0, A, B,
               M, N, K, kchunk, oo);
  if (kEpi == kEpiPartF32) {
    const long long n = 1LL * M * N;
    PISCO_KERNEL(h, k_ws_reduce, dim3(ceil_div(n, 256)), dim3(256), 0, part, nsplit, n,
                 static_cast<float*>(o.c));
  }
  return PISCO_OK;
}

HOut out16(_Float16* c, _Float16* clo, int ldc, const _Float16* bias = nullptr) {
  HOut o{};
  o.c = c;
  o.clo = clo;
  o.ldc = ldc;
  o.bias = bias;
  return o;
}

HOut out32(float* c, int ldc, const _Float16* bias = nullptr) {
  HOut o{};
  o.c = c;
  o.ldc = ldc;
  o.bias = bias;
  return o;
}

// ------------------------------------------------------------------ loss, sums, optimizer

// Per voxel: c_hat = n + y, loss 1 - |c_hat^H c|^2 / ||c_hat||^2 and its
// gradient g = -(2 / ||c_hat||^2) (conj(s) c - (|s|^2 / ||c_hat||^2) c_hat),
// s = c_hat^H c, stored as dY (N x 2Q, re / im interleaved) in two FP16
// parts hi + lo.
__global__ void k_ws_loss(const float* __restrict__ Y, const float2* __restrict__ nb,
                          const float2* __restrict__ target, int Q, long long N,
                          float* __restrict__ loss, _Float16* __restrict__ dY,
                          _Float16* __restrict__ dYlo) {
  const long long v = blockIdx.x * 256LL + threadIdx.x;
  if (v >= N) return;
  // loops over the kMaxQ bound (unrolled, guarded by q < Q) keep ch in
  // registers; a loop to Q would index it at run time, in scratch memory
  float2 ch[kMaxQ];
  float sr = 0.f, si = 0.f, nn = 0.f;
#pragma unroll
  for (int q = 0; q < kMaxQ; ++q) {
    if (q >= Q) continue;
    const float2 n = nb[size_t(q) * N + v], c = target[size_t(q) * N + v];
    const float2 a = make_float2(n.x + Y[size_t(v) * 2 * Q + 2 * q],
                                 n.y + Y[size_t(v) * 2 * Q + 2 * q + 1]);
    ch[q] = a;
    sr += a.x * c.x + a.y * c.y;  // conj(a) c
    si += a.x * c.y - a.y * c.x;
    nn += a.x * a.x + a.y * a.y;
  }
  const float s2 = sr * sr + si * si;
  const float inv = nn > 0.f ? 1.f / nn : 0.f;
  loss[v] = 1.f - s2 * inv;
#pragma unroll
  for (int q = 0; q < kMaxQ; ++q) {
    if (q >= Q) continue;
    const float2 c = target[size_t(q) * N + v];
    // conj(s) c
    const float ur = sr * c.x + si * c.y, ui = sr * c.y - si * c.x;
    const float gr = -2.f * inv * (ur - s2 * inv * ch[q].x);
    const float gi = -2.f * inv * (ui - s2 * inv * ch[q].y);
    const _Float16 hr = static_cast<_Float16>(gr), hi = static_cast<_Float16>(gi);
    dY[size_t(v) * 2 * Q + 2 * q] = hr;
    dY[size_t(v) * 2 * Q + 2 * q + 1] = hi;
    dYlo[size_t(v) * 2 * Q + 2 * q] = static_cast<_Float16>(gr - static_cast<float>(hr));
    dYlo[size_t(v) * 2 * Q + 2 * q + 1] = static_cast<_Float16>(gi - static_cast<float>(hi));
  }
}

// out[0] = scale * sum x[0..n) (one workgroup, fixed order)
__global__ void __launch_bounds__(1024) k_ws_sum(const float* __restrict__ x, long long n,
                                                 float scale, float* __restrict__ out) {
  __shared__ float red[1024];
  float s = 0.f;
  for (long long i = threadIdx.x; i < n; i += 1024) s += x[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int off = 512; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0] * scale;
}

// part[z][c] = sum over rows r of chunk z of (D[r][c] + Dlo[r][c]), an M x N
// matrix in two FP16 parts (bias gradients); block of 256 threads: 64
// columns x 4 row groups, blockIdx.y = chunk of `rows` rows
__global__ void __launch_bounds__(256) k_ws_colsum(const _Float16* __restrict__ D,
                                                   const _Float16* __restrict__ Dlo, int M,
                                                   int N, int rows, float* __restrict__ part) {
  __shared__ float red[4][64];
  const int c = blockIdx.x * 64 + (threadIdx.x & 63), g = threadIdx.x >> 6;
  const int r0 = blockIdx.y * rows, r1 = M < r0 + rows ? M : r0 + rows;
  float s = 0.f;
  if (c < N)
    for (int r = r0 + g; r < r1; r += 4)
      s += static_cast<float>(D[size_t(r) * N + c]) + static_cast<float>(Dlo[size_t(r) * N + c]);
  red[g][threadIdx.x & 63] = s;
  __syncthreads();
  if (g == 0 && c < N)
    part[size_t(blockIdx.y) * N + c] =
        red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] + red[3][threadIdx.x];
}

// Adam on the mean gradient (grad holds the batch sum): bias-corrected
// moments, master update, FP16 copy.
__global__ void k_ws_adam(float* __restrict__ master, float* __restrict__ m1,
                          float* __restrict__ m2, const float* __restrict__ grad, long long P,
                          float inv_n, float lr, float c1, float c2,
                          _Float16* __restrict__ w16) {
  const long long i = blockIdx.x * 256LL + threadIdx.x;
  if (i >= P) return;
  const float g = grad[i] * inv_n;
  const float a = 0.9f * m1[i] + 0.1f * g;
  const float b = 0.999f * m2[i] + 0.001f * g * g;
  m1[i] = a;
  m2[i] = b;
  const float w = master[i] - lr * (a * c1) / (sqrtf(b * c2) + 1e-8f);
  master[i] = w;
  w16[i] = static_cast<_Float16>(w);
}

// start vector = normalise(n + y), [Q][N] float2
__global__ void k_ws_apply(const float* __restrict__ Y, const float2* __restrict__ nb, int Q,
                           long long N, float2* __restrict__ out) {
  const long long v = blockIdx.x * 256LL + threadIdx.x;
  if (v >= N) return;
  float2 c[kMaxQ];  // in registers: loops over the kMaxQ bound, unrolled
  float nn = 0.f;
#pragma unroll
  for (int q = 0; q < kMaxQ; ++q) {
    if (q >= Q) continue;
    const float2 n = nb[size_t(q) * N + v];
    c[q] = make_float2(n.x + Y[size_t(v) * 2 * Q + 2 * q], n.y + Y[size_t(v) * 2 * Q + 2 * q + 1]);
    nn += c[q].x * c[q].x + c[q].y * c[q].y;
  }
  const float inv = nn > 0.f ? rsqrtf(nn) : 0.f;
#pragma unroll
  for (int q = 0; q < kMaxQ; ++q) {
    if (q >= Q) continue;
    out[size_t(q) * N + v] = make_float2(c[q].x * inv, c[q].y * inv);
  }
}

// Neighbour vectors: voxel (z, y, x) of the grid lr takes the coarse voxel
// floor((i - floor(lr/2)) / 2) + floor(lc/2) per dimension (lc = ceil(lr/2)),
// whose sample position is the nearest at or below, and rotates its largest
// entry (lowest index on ties) to be real and positive.
__global__ void k_ws_neighbor(const float2* __restrict__ coarse, int Q, int3 lr, int3 lc,
                              float2* __restrict__ nb) {
  const long long N = 1LL * lr.x * lr.y * lr.z;
  const long long v = blockIdx.x * 256LL + threadIdx.x;
  if (v >= N) return;
  const int ix = int(v % lr.x), iy = int((v / lr.x) % lr.y), iz = int(v / (1LL * lr.x * lr.y));
  auto parent = [](int i, int n, int m) {
    const int d = i - n / 2;
    const int k = (d >= 0 ? d / 2 : -((-d + 1) / 2)) + m / 2;
    return k < 0 ? 0 : (k >= m ? m - 1 : k);
  };
  const long long Nc = 1LL * lc.x * lc.y * lc.z;
  const long long pv = (1LL * parent(iz, lr.z, lc.z) * lc.y + parent(iy, lr.y, lc.y)) * lc.x +
                       parent(ix, lr.x, lc.x);
  float2 c[kMaxQ];  // in registers: loops over the kMaxQ bound, unrolled
  float best = -1.f;
  float2 cb = make_float2(0.f, 0.f);  // the largest entry (lowest index on ties)
#pragma unroll
  for (int q = 0; q < kMaxQ; ++q) {
    if (q >= Q) continue;
    c[q] = coarse[size_t(q) * Nc + pv];
    const float m = c[q].x * c[q].x + c[q].y * c[q].y;
    if (m > best) {
      best = m;
      cb = c[q];
    }
  }
  const float mag = sqrtf(best);
  const float2 ph = mag > 0.f ? make_float2(cb.x / mag, -cb.y / mag) : make_float2(1.f, 0.f);
#pragma unroll
  for (int q = 0; q < kMaxQ; ++q) {
    if (q >= Q) continue;
    nb[size_t(q) * N + v] = make_float2(c[q].x * ph.x - c[q].y * ph.y, c[q].x * ph.y + c[q].y * ph.x);
  }
}

// He-uniform weights (limit sqrt(6 / fan_in)), the output layer scaled by
// 1e-2 so that the untrained network returns about n; zero biases.
__global__ void k_ws_init(float* __restrict__ master, _Float16* __restrict__ w16, long long P,
                          long long off_b1, long long off_w2, long long off_b2,
                          long long off_w3, long long off_b3, int din, int h,
                          unsigned long long seed) {
  const long long i = blockIdx.x * 256LL + threadIdx.x;
  if (i >= P) return;
  unsigned long long x = seed * 0x9E3779B97F4A7C15ull + static_cast<unsigned long long>(i);
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  x ^= x >> 31;
  const float u = float(double(x >> 11) * (2.0 / 9007199254740992.0) - 1.0);
  float w = 0.f;
  if (i < off_b1) w = u * sqrtf(6.f / din);
  else if (i >= off_w2 && i < off_b2) w = u * sqrtf(6.f / h);
  else if (i >= off_w3 && i < off_b3) w = 1e-2f * u * sqrtf(6.f / h);
  master[i] = w;
  w16[i] = static_cast<_Float16>(w);
}

// out[c] = column sums of the M x N pair D + Dlo, by row chunks (partials in
// part, then k_ws_reduce, fixed order)
pisco_status_t colsum(Handle* h, const _Float16* D, const _Float16* Dlo, int M, int N,
                      float* part, float* out) {
  int chunks = ceil_div(M, 512);
  const int cap = int((1LL << 22) / N);
  if (chunks > 256) chunks = 256;
  if (chunks > cap) chunks = cap;
  if (chunks < 1) chunks = 1;
  const int rows = ceil_div(M, chunks);
  chunks = ceil_div(M, rows);
  if (chunks < 1) chunks = 1;
  PISCO_KERNEL(h, k_ws_colsum, dim3(ceil_div(N, 64), chunks), dim3(256), 0, D, Dlo, M, N, rows,
               part);
  PISCO_KERNEL(h, k_ws_reduce, dim3(ceil_div(N, 256)), dim3(256), 0, part, chunks, (long long)N,
               out);
  return PISCO_OK;
}

// Activations and per-voxel gradients in two FP16 parts each (hi, lo); the
// forward pass of inference uses the hi parts alone.
struct WsBuffers {
  _Float16 *X[2], *H1[2], *H2[2], *dY[2], *dH2[2], *dH1[2];
  float *Y, *loss, *grad, *part;
};

size_t ws_layout(const WsDims& d, long long N, void* base, WsBuffers* o) {
  Carver c(base);
  WsBuffers w{};
  for (int p = 0; p < 2; ++p) {
    w.X[p] = c.take<_Float16>(size_t(N) * d.din);
    w.H1[p] = c.take<_Float16>(size_t(N) * d.h);
    w.H2[p] = c.take<_Float16>(size_t(N) * d.h);
    w.dY[p] = c.take<_Float16>(size_t(N) * d.dout);
    w.dH2[p] = c.take<_Float16>(size_t(N) * d.h);
    w.dH1[p] = c.take<_Float16>(size_t(N) * d.h);
  }
  w.Y = c.take<float>(size_t(N) * d.dout);
  w.loss = c.take<float>(size_t(N));
  w.grad = c.take<float>(size_t(d.count));
  w.part = c.take<float>(size_t(kPartFloats));
  if (o) *o = w;
  return c.used + 256;
}

// Inference (split = false): FP16 activations.  Training (split = true):
// features and activations as hi + lo, so that the pre-activations, and
// with them the ReLU masks of the backward pass, carry FP32 accuracy
// (weights are FP16 by definition and exact in one part).
pisco_status_t ws_forward(Handle* h, const WsDims& d, long long N, float bound,
                          const float2* G, const float2* nb, const _Float16* w,
                          const WsBuffers& b, bool split) {
  const int n = int(N);
  PISCO_KERNEL(h, k_ws_features, dim3(ceil_div(N, 256)), dim3(256), 0, G, nb, d.Q, N,
               1.f / bound, b.X[0], split ? b.X[1] : nullptr);
  pisco_status_t st;
  const HOperand W1 = hop(w + d.off_w1, nullptr, d.din), W2 = hop(w + d.off_w2, nullptr, d.h),
                 W3 = hop(w + d.off_w3, nullptr, d.h);
  if (split) {
    if ((st = hgemm<true, true, 2, 1, kEpiBiasReluSplit>(
             h, hop(b.X[0], b.X[1], n), W1, n, d.h, d.din,
             out16(b.H1[0], b.H1[1], d.h, w + d.off_b1))))
      return st;
    if ((st = hgemm<false, true, 2, 1, kEpiBiasReluSplit>(
             h, hop(b.H1[0], b.H1[1], d.h), W2, n, d.h, d.h,
             out16(b.H2[0], b.H2[1], d.h, w + d.off_b2))))
      return st;
    return hgemm<false, true, 2, 1, kEpiBiasF32>(h, hop(b.H2[0], b.H2[1], d.h), W3, n, d.dout,
                                                 d.h, out32(b.Y, d.dout, w + d.off_b3));
  }
  if ((st = hgemm<true, true, 1, 1, kEpiBiasReluF16>(h, hop(b.X[0], nullptr, n), W1, n,
                                                      d.h, d.din,
                                                      out16(b.H1[0], nullptr, d.h, w + d.off_b1))))
    return st;
  if ((st = hgemm<false, true, 1, 1, kEpiBiasReluF16>(h, hop(b.H1[0], nullptr, d.h), W2, n, d.h,
                                                      d.h,
                                                      out16(b.H2[0], nullptr, d.h, w + d.off_b2))))
    return st;
  return hgemm<false, true, 1, 1, kEpiBiasF32>(h, hop(b.H2[0], nullptr, d.h), W3, n, d.dout, d.h,
                                               out32(b.Y, d.dout, w + d.off_b3));
}

// Gradient of the summed loss into b.grad (FP32, parameter layout), from the
// split forward pass and dY; weight gradients by split K over the voxels.
pisco_status_t ws_backward(Handle* h, const WsDims& d, long long N, const _Float16* w,
                           const WsBuffers& b) {
  const int n = int(N);
  pisco_status_t st;
  const HOperand dYk = hop(b.dY[0], b.dY[1], d.dout), H2 = hop(b.H2[0], b.H2[1], d.h),
                 H1 = hop(b.H1[0], b.H1[1], d.h), X = hop(b.X[0], b.X[1], n),
                 dH2 = hop(b.dH2[0], b.dH2[1], d.h), dH1 = hop(b.dH1[0], b.dH1[1], d.h);
  // dW3 = dY^T H2, db3 = column sums of dY
  if ((st = hgemm<true, false, 2, 2, kEpiPartF32>(h, dYk, H2, d.dout, d.h, n,
                                                  out32(b.grad + d.off_w3, d.h), b.part)))
    return st;
  if ((st = colsum(h, b.dY[0], b.dY[1], n, d.dout, b.part, b.grad + d.off_b3))) return st;
  // dH2 = (dY W3) masked by h2 > 0
  HOut m2 = out16(b.dH2[0], b.dH2[1], d.h);
  m2.mask[0] = b.H2[0];
  m2.mask[1] = b.H2[1];
  m2.ldm = d.h;
  if ((st = hgemm<false, false, 2, 1, kEpiMaskSplit>(h, dYk, hop(w + d.off_w3, nullptr, d.h), n,
                                                     d.h, d.dout, m2)))
    return st;
  if ((st = hgemm<true, false, 2, 2, kEpiPartF32>(h, dH2, H1, d.h, d.h, n,
                                                  out32(b.grad + d.off_w2, d.h), b.part)))
    return st;
  if ((st = colsum(h, b.dH2[0], b.dH2[1], n, d.h, b.part, b.grad + d.off_b2))) return st;
  HOut m1 = out16(b.dH1[0], b.dH1[1], d.h);
  m1.mask[0] = b.H1[0];
  m1.mask[1] = b.H1[1];
  m1.ldm = d.h;
  if ((st = hgemm<false, false, 2, 1, kEpiMaskSplit>(h, dH2, hop(w + d.off_w2, nullptr, d.h), n,
                                                     d.h, d.h, m1)))
    return st;
  if ((st = hgemm<true, true, 2, 2, kEpiPartF32>(h, dH1, X, d.h, d.din, n,
                                                  out32(b.grad + d.off_w1, d.din), b.part)))
    return st;
  if ((st = colsum(h, b.dH1[0], b.dH1[1], n, d.h, b.part, b.grad + d.off_b1))) return st;
  return PISCO_OK;
}

pisco_status_t ws_check(Handle* h, int Q, long long N) {
  if (!h) return PISCO_ERR_ARG;
  if (Q < 2 || Q > kMaxQ) {
    h->last_error = "warm start: Q must be in [2, 32]";
    return PISCO_ERR_ARG;
  }
  if (N < 0 || N > (1LL << 31) / (Q * Q + 2 * Q)) {
    h->last_error = "warm start: N out of range";
    return PISCO_ERR_ARG;
  }
  return PISCO_OK;
}

}  // namespace

}  // namespace pisco

using namespace pisco;

extern "C" {

pisco_status_t pisco_ws_param_count(int32_t Q, int64_t* count) {
  if (Q < 2 || Q > kMaxQ || !count) return PISCO_ERR_ARG;
  *count = ws_dims(Q).count;
  return PISCO_OK;
}

pisco_status_t pisco_ws_workspace_size(int32_t Q, int64_t N, size_t* bytes) {
  if (Q < 2 || Q > kMaxQ || N < 0 || !bytes) return PISCO_ERR_ARG;
  *bytes = ws_layout(ws_dims(Q), N, nullptr, nullptr);
  return PISCO_OK;
}

pisco_status_t pisco_ws_init(pisco_handle_t handle, int32_t Q, uint64_t seed, float* master,
                             void* weights16) {
  Handle* h = reinterpret_cast<Handle*>(handle);
  pisco_status_t st = ws_check(h, Q, 0);
  if (st) return st;
  if (!master || !weights16) {
    h->last_error = "warm start: null pointer";
    return PISCO_ERR_ARG;
  }
  const WsDims d = ws_dims(Q);
  PISCO_KERNEL(h, k_ws_init, dim3(ceil_div(d.count, 256)), dim3(256), 0, master,
               static_cast<_Float16*>(weights16), d.count, d.off_b1, d.off_w2, d.off_b2,
               d.off_w3, d.off_b3, d.din, d.h, static_cast<unsigned long long>(seed));
  return PISCO_OK;
}

pisco_status_t pisco_ws_neighbor(pisco_handle_t handle, int32_t Q, const int32_t grid_lr[3],
                                 const void* coarse, void* neighbor) {
  Handle* h = reinterpret_cast<Handle*>(handle);
  pisco_status_t st = ws_check(h, Q, 0);
  if (st) return st;
  if (!grid_lr || !coarse || !neighbor || grid_lr[0] < 1 || grid_lr[1] < 1 || grid_lr[2] < 1) {
    h->last_error = "warm start: bad neighbour arguments";
    return PISCO_ERR_ARG;
  }
  const int3 lr = make_int3(grid_lr[2], grid_lr[1], grid_lr[0]);
  const int3 lc = make_int3((lr.x + 1) / 2, (lr.y + 1) / 2, (lr.z + 1) / 2);
  const long long N = 1LL * lr.x * lr.y * lr.z;
  PISCO_KERNEL(h, k_ws_neighbor, dim3(ceil_div(N, 256)), dim3(256), 0,
               static_cast<const float2*>(coarse), Q, lr, lc, static_cast<float2*>(neighbor));
  return PISCO_OK;
}

pisco_status_t pisco_ws_forward(pisco_handle_t handle, int32_t Q, int64_t N, float bound,
                                const void* G, const void* neighbor, const void* weights16,
                                void* init, void* ws, size_t ws_bytes) {
  Handle* h = reinterpret_cast<Handle*>(handle);
  pisco_status_t st = ws_check(h, Q, N);
  if (st) return st;
  if (N == 0) return PISCO_OK;
  if (!G || !neighbor || !weights16 || !init || !ws || !(bound > 0.f)) {
    h->last_error = "warm start: null pointer or bad bound";
    return PISCO_ERR_ARG;
  }
  const WsDims d = ws_dims(Q);
  if (ws_bytes < ws_layout(d, N, nullptr, nullptr)) {
    h->last_error = "warm start: workspace too small";
    return PISCO_ERR_WORKSPACE;
  }
  WsBuffers b;
  ws_layout(d, N, ws, &b);
  const _Float16* w = static_cast<const _Float16*>(weights16);
  const float2* nb = static_cast<const float2*>(neighbor);
  if ((st = ws_forward(h, d, N, bound, static_cast<const float2*>(G), nb, w, b, false)))
    return st;
  PISCO_KERNEL(h, k_ws_apply, dim3(ceil_div(N, 256)), dim3(256), 0, b.Y, nb, Q, N,
               static_cast<float2*>(init));
  return PISCO_OK;
}

pisco_status_t pisco_ws_train_step(pisco_handle_t handle, int32_t Q, int64_t N, float bound,
                                   const void* G, const void* neighbor, const void* target,
                                   float* master, void* weights16, float* adam_m,
                                   float* adam_v, int32_t step, float lr, float* loss_out,
                                   float* grad_out, void* ws, size_t ws_bytes) {
  Handle* h = reinterpret_cast<Handle*>(handle);
  pisco_status_t st = ws_check(h, Q, N);
  if (st) return st;
  if (N < 1 || !G || !neighbor || !target || !weights16 || !ws || !(bound > 0.f) ||
      (step > 0 && (!master || !adam_m || !adam_v))) {
    h->last_error = "warm start: null pointer, empty batch or bad bound";
    return PISCO_ERR_ARG;
  }
  const WsDims d = ws_dims(Q);
  if (ws_bytes < ws_layout(d, N, nullptr, nullptr)) {
    h->last_error = "warm start: workspace too small";
    return PISCO_ERR_WORKSPACE;
  }
  WsBuffers b;
  ws_layout(d, N, ws, &b);
  _Float16* w = static_cast<_Float16*>(weights16);
  const float2* nb = static_cast<const float2*>(neighbor);
  if ((st = ws_forward(h, d, N, bound, static_cast<const float2*>(G), nb, w, b, true)))
    return st;
  PISCO_KERNEL(h, k_ws_loss, dim3(ceil_div(N, 256)), dim3(256), 0, b.Y, nb,
               static_cast<const float2*>(target), Q, N, b.loss, b.dY[0], b.dY[1]);
  if (loss_out)
    PISCO_KERNEL(h, k_ws_sum, dim3(1), dim3(1024), 0, b.loss, N, float(1.0 / double(N)), loss_out);
  if ((st = ws_backward(h, d, N, w, b))) return st;
  if (grad_out) {
    hipError_t e = hipMemcpyAsync(grad_out, b.grad, sizeof(float) * size_t(d.count),
                                  hipMemcpyDeviceToDevice, h->stream);
    if (e != hipSuccess) return hip_check(h, e, "warm start gradient copy");
  }
  if (step > 0) {
    const double c1 = 1.0 / (1.0 - std::pow(0.9, step));
    const double c2 = 1.0 / (1.0 - std::pow(0.999, step));
    PISCO_KERNEL(h, k_ws_adam, dim3(ceil_div(d.count, 256)), dim3(256), 0, master, adam_m,
                 adam_v, b.grad, d.count, float(1.0 / double(N)), lr, float(c1), float(c2), w);
  }
  return PISCO_OK;
}

}  // extern "C"
