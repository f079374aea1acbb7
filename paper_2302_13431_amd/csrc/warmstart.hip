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
// Arithmetic: weights and activations FP16, products on the matrix cores
// (v_mfma_f32_16x16x16f16) with FP32 accumulation; per-voxel gradients FP16
// (they are O(1): the batch mean is applied to the FP32 weight gradients);
// loss, weight gradients and optimizer state FP32.
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

typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));
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

// X[v][j] (FP16, row-major N x Din) from packed G ([pair][N] float2) and the
// neighbour vectors ([Q][N] float2).
__global__ void k_ws_features(const float2* __restrict__ G, const float2* __restrict__ nb,
                              int Q, long long N, float inv_bound, _Float16* __restrict__ X) {
  const int din = Q * Q + 2 * Q;
  const long long idx = blockIdx.x * 256LL + threadIdx.x;
  if (idx >= N * din) return;
  const long long v = idx / din;
  const int j = int(idx - v * din);
  float f;
  if (j < Q) {
    f = G[size_t(pair_index(j, j, Q)) * N + v].x * inv_bound;
  } else if (j < Q * Q) {
    // off-diagonal entry o in row-major order of p < q, then re / im
    int o = (j - Q) >> 1, p = 0;
    while (o >= Q - 1 - p) {
      o -= Q - 1 - p;
      ++p;
    }
    const float2 g = G[size_t(pair_index(p, p + 1 + o, Q)) * N + v];
    f = ((j - Q) & 1 ? g.y : g.x) * inv_bound;
  } else {
    const int k = j - Q * Q;
    const float2 n = nb[size_t(k >> 1) * N + v];
    f = k & 1 ? n.y : n.x;
  }
  X[idx] = static_cast<_Float16>(f);
}

// ------------------------------------------------------------------ GEMM

// C (M x N) = op(A) (M x K) op(B) (K x N), FP16 operands, FP32 accumulation
// on the matrix cores.  op(A)(m, k) = kTA ? A[k lda + m] : A[m lda + k];
// op(B)(k, n) = kTB ? B[n ldb + k] : B[k ldb + n].  Workgroup tile 64 x 64,
// four waves of 32 x 32 (2 x 2 blocks of 16 x 16), K in steps of 16.
// Operand lanes: lane l holds row (column) l % 16 at k = 4 (l / 16) + j;
// accumulator element v of lane l is row 4 (l / 16) + v, column l % 16.
// Epilogues:
enum : int {
  kEpiBiasReluF16 = 0,  // C16 = fp16(max(acc + bias[n], 0)), bias FP16
  kEpiBiasF32 = 1,      // C32 = acc + bias[n], bias FP16
  kEpiMaskF16 = 2,      // C16 = fp16(acc) where mask16[m][n] > 0, else 0
  kEpiF32 = 3,          // C32 = acc
};

template <bool kTA, bool kTB, int kEpi>
__global__ void __launch_bounds__(256) k_hgemm(const _Float16* __restrict__ A, int lda,
                                               const _Float16* __restrict__ B, int ldb, int M,
                                               int N, int K, const _Float16* __restrict__ bias,
                                               const _Float16* __restrict__ mask, int ldm,
                                               void* __restrict__ C, int ldc) {
  const int t = threadIdx.x, wv = t >> 6, l = t & 63;
  const int li = l & 15, kg = l >> 4;
  const int m0 = blockIdx.x * 64 + (wv & 1) * 32, n0 = blockIdx.y * 64 + (wv >> 1) * 32;
  f32x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < K; k0 += 16) {
    f16x4 a[2], b[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int m = m0 + 16 * i + li;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int k = k0 + 4 * kg + j;
        _Float16 v = 0;
        if (m < M && k < K) v = kTA ? A[size_t(k) * lda + m] : A[size_t(m) * lda + k];
        a[i][j] = v;
      }
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int n = n0 + 16 * i + li;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int k = k0 + 4 * kg + j;
        _Float16 v = 0;
        if (n < N && k < K) v = kTB ? B[size_t(n) * ldb + k] : B[size_t(k) * ldb + n];
        b[i][j] = v;
      }
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16f16(a[i], b[j], acc[i][j], 0, 0, 0);
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int m = m0 + 16 * i + 4 * kg + v, n = n0 + 16 * j + li;
        if (m >= M || n >= N) continue;
        const float x = acc[i][j][v];
        if (kEpi == kEpiBiasReluF16) {
          static_cast<_Float16*>(C)[size_t(m) * ldc + n] =
              static_cast<_Float16>(fmaxf(x + static_cast<float>(bias[n]), 0.f));
        } else if (kEpi == kEpiBiasF32) {
          static_cast<float*>(C)[size_t(m) * ldc + n] = x + static_cast<float>(bias[n]);
        } else if (kEpi == kEpiMaskF16) {
          const bool on = static_cast<float>(mask[size_t(m) * ldm + n]) > 0.f;
          static_cast<_Float16*>(C)[size_t(m) * ldc + n] = static_cast<_Float16>(on ? x : 0.f);
        } else {
          static_cast<float*>(C)[size_t(m) * ldc + n] = x;
        }
      }
}

template <bool kTA, bool kTB, int kEpi>
pisco_status_t hgemm(Handle* h, const _Float16* A, int lda, const _Float16* B, int ldb, int M,
                     int N, int K, const _Float16* bias, const _Float16* mask, int ldm, void* C,
                     int ldc) {
  if (M <= 0 || N <= 0) return PISCO_OK;
  dim3 g(ceil_div(M, 64), ceil_div(N, 64));
  PISCO_KERNEL(h, (k_hgemm<kTA, kTB, kEpi>), g, dim3(256), 0, A, lda, B, ldb, M, N, K, bias,
               mask, ldm, C, ldc);
  return PISCO_OK;
}

// ------------------------------------------------------------------ loss, sums, optimizer

// Per voxel: c_hat = n + y, loss 1 - |c_hat^H c|^2 / ||c_hat||^2 and its
// gradient g = -(2 / ||c_hat||^2) (conj(s) c - (|s|^2 / ||c_hat||^2) c_hat),
// s = c_hat^H c, stored as dY (FP16, N x 2Q, re / im interleaved).
__global__ void k_ws_loss(const float* __restrict__ Y, const float2* __restrict__ nb,
                          const float2* __restrict__ target, int Q, long long N,
                          float* __restrict__ loss, _Float16* __restrict__ dY) {
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
    dY[size_t(v) * 2 * Q + 2 * q] = static_cast<_Float16>(gr);
    dY[size_t(v) * 2 * Q + 2 * q + 1] = static_cast<_Float16>(gi);
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

// out[c] = sum_r D[r][c] for an M x N FP16 matrix (bias gradients); block of
// 256 threads: 64 columns x 4 row groups
__global__ void __launch_bounds__(256) k_ws_colsum(const _Float16* __restrict__ D, int M,
                                                   int N, float* __restrict__ out) {
  __shared__ float red[4][64];
  const int c = blockIdx.x * 64 + (threadIdx.x & 63), g = threadIdx.x >> 6;
  float s = 0.f;
  if (c < N)
    for (int r = g; r < M; r += 4) s += static_cast<float>(D[size_t(r) * N + c]);
  red[g][threadIdx.x & 63] = s;
  __syncthreads();
  if (g == 0 && c < N)
    out[c] = red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] + red[3][threadIdx.x];
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

struct WsBuffers {
  _Float16 *X, *H1, *H2, *dY, *dH2, *dH1;
  float *Y, *loss, *grad;
};

size_t ws_layout(const WsDims& d, long long N, void* base, WsBuffers* o) {
  Carver c(base);
  WsBuffers w{};
  w.X = c.take<_Float16>(size_t(N) * d.din);
  w.H1 = c.take<_Float16>(size_t(N) * d.h);
  w.H2 = c.take<_Float16>(size_t(N) * d.h);
  w.Y = c.take<float>(size_t(N) * d.dout);
  w.dY = c.take<_Float16>(size_t(N) * d.dout);
  w.dH2 = c.take<_Float16>(size_t(N) * d.h);
  w.dH1 = c.take<_Float16>(size_t(N) * d.h);
  w.loss = c.take<float>(size_t(N));
  w.grad = c.take<float>(size_t(d.count));
  if (o) *o = w;
  return c.used + 256;
}

pisco_status_t ws_forward(Handle* h, const WsDims& d, long long N, float bound,
                          const float2* G, const float2* nb, const _Float16* w,
                          const WsBuffers& b) {
  const int n = int(N);
  PISCO_KERNEL(h, k_ws_features, dim3(ceil_div(N * d.din, 256)), dim3(256), 0, G, nb, d.Q, N,
               1.f / bound, b.X);
  pisco_status_t st;
  if ((st = hgemm<false, true, kEpiBiasReluF16>(h, b.X, d.din, w + d.off_w1, d.din, n, d.h,
                                                d.din, w + d.off_b1, nullptr, 0, b.H1, d.h)))
    return st;
  if ((st = hgemm<false, true, kEpiBiasReluF16>(h, b.H1, d.h, w + d.off_w2, d.h, n, d.h, d.h,
                                                w + d.off_b2, nullptr, 0, b.H2, d.h)))
    return st;
  return hgemm<false, true, kEpiBiasF32>(h, b.H2, d.h, w + d.off_w3, d.h, n, d.dout, d.h,
                                         w + d.off_b3, nullptr, 0, b.Y, d.dout);
}

// Gradient of the summed loss into b.grad (FP32, parameter layout).
pisco_status_t ws_backward(Handle* h, const WsDims& d, long long N, const _Float16* w,
                           const WsBuffers& b) {
  const int n = int(N);
  pisco_status_t st;
  if ((st = hgemm<true, false, kEpiF32>(h, b.dY, d.dout, b.H2, d.h, d.dout, d.h, n, nullptr,
                                        nullptr, 0, b.grad + d.off_w3, d.h)))
    return st;
  PISCO_KERNEL(h, k_ws_colsum, dim3(ceil_div(d.dout, 64)), dim3(256), 0, b.dY, n, d.dout, b.grad + d.off_b3);
  if ((st = hgemm<false, false, kEpiMaskF16>(h, b.dY, d.dout, w + d.off_w3, d.h, n, d.h, d.dout,
                                             nullptr, b.H2, d.h, b.dH2, d.h)))
    return st;
  if ((st = hgemm<true, false, kEpiF32>(h, b.dH2, d.h, b.H1, d.h, d.h, d.h, n, nullptr, nullptr,
                                        0, b.grad + d.off_w2, d.h)))
    return st;
  PISCO_KERNEL(h, k_ws_colsum, dim3(ceil_div(d.h, 64)), dim3(256), 0, b.dH2, n, d.h, b.grad + d.off_b2);
  if ((st = hgemm<false, false, kEpiMaskF16>(h, b.dH2, d.h, w + d.off_w2, d.h, n, d.h, d.h,
                                             nullptr, b.H1, d.h, b.dH1, d.h)))
    return st;
  if ((st = hgemm<true, false, kEpiF32>(h, b.dH1, d.h, b.X, d.din, d.h, d.din, n, nullptr,
                                        nullptr, 0, b.grad + d.off_w1, d.din)))
    return st;
  PISCO_KERNEL(h, k_ws_colsum, dim3(ceil_div(d.h, 64)), dim3(256), 0, b.dH1, n, d.h, b.grad + d.off_b1);
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
  if ((st = ws_forward(h, d, N, bound, static_cast<const float2*>(G), nb, w, b))) return st;
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
  if ((st = ws_forward(h, d, N, bound, static_cast<const float2*>(G), nb, w, b))) return st;
  PISCO_KERNEL(h, k_ws_loss, dim3(ceil_div(N, 256)), dim3(256), 0, b.Y, nb,
               static_cast<const float2*>(target), Q, N, b.loss, b.dY);
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
