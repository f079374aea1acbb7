// Calibration Gram C^H C by zero-padded FFT correlation (Sec. IV-A).
//
// Column i of C_p^H C_q is a shift of the single correlation
//   R_pq[d] = sum_k conj(s_p[k]) s_q[k + d]
// so the whole Gram follows from Q forward FFTs of the zero-padded channels,
// one cross-spectrum and one inverse FFT per channel pair, and a gather.  The
// pad F >= A + 2 tau per dimension makes the circular correlation equal the
// linear one at every lag |d| <= 2 tau that the gather needs.
//
// Only the Q(Q+1)/2 pairs p <= q are transformed; the lower blocks are the
// conjugate transpose of the upper ones, which also makes the result exactly
// Hermitian.  Transforms are separable passes of radix-2 Stockham FFTs held in
// LDS; the forward passes skip the zero padding on input and the inverse passes
// keep only the 4 tau + 1 lags per dimension on output.
#include <cstdio>
#include <mutex>

#include "common.hpp"

namespace pisco {

// Library-owned scratch of pisco_gram_static (for callers that cannot
// allocate): one copy per GPU, held until the process ends.  Host code uses
// the per-device address from hipGetSymbolAddress, never the array's name.
static __device__ __align__(256) char scratch[kGramScratchBytes];

namespace {
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

pisco_status_t gram_scratch_address(Handle* h, void** out) {
  *out = nullptr;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_check(h, e, "scratch: current device");
  if (dev < 0 || dev >= kMaxDevices) {
    if (h) h->last_error = "scratch: device index out of range";
    return PISCO_ERR_UNSUPPORTED;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_check(h, e, "scratch: symbol address");
    if (!ptr) {
      if (h) h->last_error = "scratch: null symbol address";
      return PISCO_ERR_HIP;
    }
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return PISCO_OK;
}

// In-LDS radix-2 Stockham FFT of LPB lines of length L, stored line-major in
// `a` (scratch `b` of the same size).  Thread t handles butterfly `bt` of line
// `ln`.  sign = -1: e^{-i 2 pi f k / L}; sign = +1: e^{+i ...} (unnormalised).
// Every thread of the block must call this (it synchronises the block).
__device__ float2* lds_fft(float2* a, float2* b, int L, int ln, int bt, bool active,
                           float sign) {
  const int half = L >> 1;
  for (int ns = 1; ns < L; ns <<= 1) {
    if (active) {
      float2* x = a + ln * L;
      float2* y = b + ln * L;
      for (int j = bt; j < half; j += 128) {
        const int k = j & (ns - 1);
        float sn, cs;
        sincospif(sign * float(k) / float(ns), &sn, &cs);
        const float2 u = x[j];
        const float2 v = cmul(x[j + half], make_float2(cs, sn));
        const int o = ((j - k) << 1) + k;
        y[o] = cadd(u, v);
        y[o + ns] = csub(u, v);
      }
    }
    __syncthreads();
    float2* t = a;
    a = b;
    b = t;
  }
  return a;
}

// Maps FFT position j (0..F-1) of a zero-padded, centred sequence of A samples
// to the array index a (k = a - floor(A/2), j = k mod F); -1 if padding.
__device__ inline int pad_source(int j, int A, int F) {
  const int h = A / 2;
  int k = (j <= A - 1 - h) ? j : j - F;
  if (k < -h || k > A - 1 - h) return -1;
  return k + h;
}

// Lag kept at output slot m (0..B-1) of an inverse pass: d = m - (B-1)/2,
// found at FFT position d mod F.
__device__ inline int lag_position(int m, int B, int F) {
  int d = m - (B - 1) / 2;
  return d < 0 ? d + F : d;
}

__device__ inline void pair_decode(int pair, int Q, int* p, int* q) {
  int base = 0;
  for (int pp = 0; pp < Q; ++pp) {
    const int cnt = Q - pp;
    if (pair < base + cnt) {
      *p = pp;
      *q = pp + (pair - base);
      return;
    }
    base += cnt;
  }
  *p = Q - 1;
  *q = Q - 1;
}

struct PassGeom {
  int L;        // FFT length
  int nlines;
  int lpb;      // lines per block
  int thr;      // threads per line (= min(L/2, 128))
};

static PassGeom geom(int L, long long nlines) {
  PassGeom g;
  g.L = L;
  g.thr = L / 2 < 128 ? (L / 2 > 0 ? L / 2 : 1) : 128;
  g.lpb = 256 / g.thr;
  g.nlines = int(nlines);
  return g;
}

// Thread-to-(line, butterfly) mapping.  When the lines are contiguous in
// memory (the x passes), consecutive threads walk along a line; otherwise
// consecutive threads take consecutive lines so global accesses coalesce.
template <bool kAlongLine>
__device__ inline void map_thread(const PassGeom& g, int* ln, int* bt) {
  const int t = threadIdx.x;
  if (kAlongLine) {
    *ln = t / g.thr;
    *bt = t % g.thr;
  } else {
    *ln = t % g.lpb;
    *bt = t / g.lpb;
  }
}

// ---------------------------------------------------------------- forward passes

// x pass: lines (q, az, ay) of the ACS, zero-padded to F2 -> S1[q][az][ay][F2]
__global__ void __launch_bounds__(256) k_fwd_x(const float2* __restrict__ acs,
                                               float2* __restrict__ out, PassGeom g,
                                               int A2, int F2, unsigned* status) {
  __shared__ float2 sa[2 * 256 * 2];
  float2* a = sa;
  float2* b = sa + 2 * 256;
  int ln, bt;
  map_thread<true>(g, &ln, &bt);
  const int line = blockIdx.x * g.lpb + ln;
  const bool active = line < g.nlines && ln < g.lpb;
  if (active) {
    for (int j = bt; j < g.L; j += g.thr) {
      const int src = pad_source(j, A2, F2);
      float2 v = make_float2(0.f, 0.f);
      if (src >= 0) {
        v = acs[size_t(line) * A2 + src];
        if (!isfinite(v.x) || !isfinite(v.y)) {
          atomicOr(status, PISCO_FLAG_NONFINITE);
          v = make_float2(0.f, 0.f);
        }
      }
      a[ln * g.L + j] = v;
    }
  }
  __syncthreads();
  float2* r = lds_fft(a, b, g.L, ln, bt, active, -1.f);
  if (active)
    for (int j = bt; j < g.L; j += g.thr) out[size_t(line) * F2 + j] = r[ln * g.L + j];
}

// y or z pass over a [outer][A][inner] array: lines (outer, inner), the A
// samples along the middle axis are zero-padded to F -> [outer][F][inner]
__global__ void __launch_bounds__(256) k_fwd_mid(const float2* __restrict__ in,
                                                 float2* __restrict__ out, PassGeom g,
                                                 int A, int F, int inner) {
  __shared__ float2 sa[2 * 256 * 2];
  float2* a = sa;
  float2* b = sa + 2 * 256;
  int ln, bt;
  map_thread<false>(g, &ln, &bt);
  const int line = blockIdx.x * g.lpb + ln;
  const bool active = line < g.nlines;
  const int outer = active ? line / inner : 0, in_i = active ? line % inner : 0;
  if (active) {
    for (int j = bt; j < g.L; j += g.thr) {
      const int src = pad_source(j, A, F);
      a[ln * g.L + j] = src >= 0 ? in[(size_t(outer) * A + src) * inner + in_i]
                                 : make_float2(0.f, 0.f);
    }
  }
  __syncthreads();
  float2* r = lds_fft(a, b, g.L, ln, bt, active, -1.f);
  if (active)
    for (int j = bt; j < g.L; j += g.thr)
      out[(size_t(outer) * F + j) * inner + in_i] = r[ln * g.L + j];
}

// ---------------------------------------------------------------- inverse passes

// First inverse pass along the slowest used axis (length F, extent of the
// axis in S), with the cross-spectrum conj(S_p) S_q formed on load.
//   S : [Q][Fa][inner];  out: [P][B][inner]; lines (pair, inner)
__global__ void __launch_bounds__(256) k_inv_first(const float2* __restrict__ S,
                                                   float2* __restrict__ out, PassGeom g,
                                                   int Q, int F, int inner, int B) {
  __shared__ float2 sa[2 * 256 * 2];
  float2* a = sa;
  float2* b = sa + 2 * 256;
  int ln, bt;
  map_thread<false>(g, &ln, &bt);
  const int line = blockIdx.x * g.lpb + ln;
  const bool active = line < g.nlines;
  int pair = 0, in_i = 0, p = 0, q = 0;
  if (active) {
    pair = line / inner;
    in_i = line % inner;
    pair_decode(pair, Q, &p, &q);
    const float2* Sp = S + size_t(p) * F * inner;
    const float2* Sq = S + size_t(q) * F * inner;
    for (int j = bt; j < g.L; j += g.thr) {
      const size_t o = size_t(j) * inner + in_i;
      a[ln * g.L + j] = cmulc(Sp[o], Sq[o]);
    }
  }
  __syncthreads();
  float2* r = lds_fft(a, b, g.L, ln, bt, active, +1.f);
  if (active)
    for (int m = bt; m < B; m += g.thr)
      out[(size_t(pair) * B + m) * inner + in_i] = r[ln * g.L + lag_position(m, B, F)];
}

// Value of lane (lane ^ h) of the wave, h a power of two below 64, on the
// ALU's data-parallel moves where one exists: quad permutations [1,0,3,2]
// (h = 1) and [2,3,0,1] (h = 2); h = 8 a rotation by 8 within 16-lane rows;
// h = 4 rotations by 12 and 4 within the row (lane + 4 and lane - 4), taken
// by lane bit 2; h = 16 a swizzle xor within 32-lane halves; h = 32 through
// the LDS crossbar.
template <int kCtrl>
__device__ inline float dpp_mov(float v) {
  return __builtin_bit_cast(
      float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), kCtrl, 0xF, 0xF, false));
}
__device__ inline float lane_xor(float v, int h, int lane) {
  switch (h) {
    case 1: return dpp_mov<0xB1>(v);
    case 2: return dpp_mov<0x4E>(v);
    case 4: {
      const float up = dpp_mov<0x12C>(v), down = dpp_mov<0x124>(v);
      return (lane & 4) ? down : up;
    }
    case 8: return dpp_mov<0x128>(v);
    case 16:
      return __builtin_bit_cast(float,
                                __builtin_amdgcn_ds_swizzle(__builtin_bit_cast(int, v), 0x401F));
    default: return __shfl_xor(v, h, 64);
  }
}

// Lane-parallel inverse transform of kIlp lines per lane (F <= 64, 64 / F
// lines per wave, lane = sub-line * F + jl): x holds the input at position
// bit-reverse(jl) and on return output position jl; tw[s] is the lane's
// twiddle e^{+i pi (jl mod h) / h} of step h = 2^s.
template <int kIlp>
__device__ inline void lane_ifft(float2 (&x)[kIlp], const float2 (&tw)[6], int F, int jl,
                                 int lane) {
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    const int h = 1 << s;
    if (h < F) {
      // the upper lane twiddles its own value and sends it, the lower lane
      // sends its value as is: lower x + W x', upper x - W x'
      const bool lo = (jl & h) == 0;
#pragma unroll
      for (int u = 0; u < kIlp; ++u) {
        const float2 w = cmul(tw[s], x[u]);
        const float2 snd = lo ? x[u] : w;
        const float2 r = make_float2(lane_xor(snd.x, h, lane), lane_xor(snd.y, h, lane));
        x[u] = lo ? cadd(x[u], r) : csub(r, w);
      }
    }
  }
}

__device__ inline void lane_twiddles(float2 (&tw)[6], int F, int jl) {
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    const int h = 1 << s;
    float sn = 0.f, cs = 1.f;
    if (h < F) sincospif(float(jl & (h - 1)) / float(h), &sn, &cs);
    tw[s] = make_float2(cs, sn);
  }
}

// First inverse pass in column blocks (F <= 64): a workgroup takes C
// consecutive columns (inner indices) of every channel's spectrum into LDS,
// laid out [q][c][j] with the F frequencies contiguous, so that each spectrum
// is read from HBM once, and forms every channel pair's cross-spectrum from
// there (the line-per-pair form re-reads two channel planes per pair).  A
// wave transforms 64 / F lines at a time across its lanes: the input in
// bit-reversed order, then radix-2 steps h = 1, 2, .., F/2 pairing lane j
// with lane j ^ h: the lower lane forms a + W b, the upper a - W b (a, b the
// lower and upper values, W = e^{+i pi (j mod h) / h}); lane j then holds
// output position j (lag j, or j - F past F/2), and the lanes at the B kept
// lags store.  A wave takes every nw-th pair of the workgroup's pair range
// (gridDim.y ranges) and its C columns in turn.
__global__ void __launch_bounds__(512) k_inv_first_cols(const float2* __restrict__ S,
                                                        float2* __restrict__ out, int Q, int F,
                                                        int logF, int inner, int B, int C) {
  extern __shared__ float2 sl[];  // [Q][C][F]
  const long long c0 = 1LL * blockIdx.x * C;
  for (int e = threadIdx.x; e < Q * F * C; e += blockDim.x) {
    const int c = e % C, j = (e / C) % F, q = e / (C * F);
    sl[(q * C + c) * F + j] =
        c0 + c < inner ? S[(size_t(q) * F + j) * inner + c0 + c] : make_float2(0.f, 0.f);
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int per = 64 / F, sub = lane / F, jl = lane % F;
  const int jr = logF > 0 ? int(__brev(unsigned(jl)) >> (32 - logF)) : 0;
  float2 tw[6];
  lane_twiddles(tw, F, jl);
  const int hb = (B - 1) / 2;
  const int m = jl <= hb ? jl + hb : (jl >= F - hb ? jl - F + hb : -1);
  // pairs [pb, pe) of this workgroup (blockIdx.y of gridDim.y groups)
  const int P = Q * (Q + 1) / 2;
  const int per_group = (P + gridDim.y - 1) / gridDim.y;
  const int pb = blockIdx.y * per_group, pe = pb + per_group < P ? pb + per_group : P;
  // kIlp lines per lane in flight, so that the cross-lane exchanges of one
  // line overlap those of the others
  constexpr int kIlp = 4;
  for (int pair = pb + wv; pair < pe; pair += nw) {
    int p, q;
    pair_decode(pair, Q, &p, &q);
    for (int cb = 0; cb < C; cb += per * kIlp) {
      float2 x[kIlp];
#pragma unroll
      for (int u = 0; u < kIlp; ++u) {
        const int c = cb + sub + per * u;
        x[u] = c < C ? cmulc(sl[(p * C + c) * F + jr], sl[(q * C + c) * F + jr])
                     : make_float2(0.f, 0.f);
      }
      lane_ifft(x, tw, F, jl, lane);
#pragma unroll
      for (int u = 0; u < kIlp; ++u) {
        const int c = cb + sub + per * u;
        if (c < C && m >= 0 && c0 + c < inner)
          out[(size_t(pair) * B + m) * inner + c0 + c] = x[u];
      }
    }
  }
}

// Middle inverse pass in column blocks (F <= 64): a workgroup takes one outer
// index and C <= 64 consecutive columns, stages the F x C input tile in LDS
// by whole rows (transposed to [c][j], rows padded by one), transforms the
// C lines across lanes as k_inv_first_cols does, and writes the B kept lags
// back through LDS as whole rows of C columns.
__global__ void __launch_bounds__(512) k_inv_mid_cols(const float2* __restrict__ in,
                                                      float2* __restrict__ out, int F, int logF,
                                                      int inner, int B, int C) {
  __shared__ float2 xin[64 * 65];  // [c][j], row stride F + 1
  __shared__ float2 xo[64 * 64];   // [m][c], row stride C
  const int cblocks = (inner + C - 1) / C;
  const long long o = blockIdx.x / cblocks;
  const int c0 = int(blockIdx.x % cblocks) * C;
  const int FS = F + 1;
  const float2* src = in + size_t(o) * F * inner;
  for (int e = threadIdx.x; e < F * C; e += blockDim.x) {
    const int j = e / C, c = e - j * C;
    xin[c * FS + j] = c0 + c < inner ? src[size_t(j) * inner + c0 + c] : make_float2(0.f, 0.f);
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int per = 64 / F, sub = lane / F, jl = lane % F;
  const int jr = logF > 0 ? int(__brev(unsigned(jl)) >> (32 - logF)) : 0;
  float2 tw[6];
  lane_twiddles(tw, F, jl);
  const int hb = (B - 1) / 2;
  const int m = jl <= hb ? jl + hb : (jl >= F - hb ? jl - F + hb : -1);
  constexpr int kIlp = 4;
  for (int cb = wv * per * kIlp; cb < C; cb += nw * per * kIlp) {
    float2 x[kIlp];
#pragma unroll
    for (int u = 0; u < kIlp; ++u) {
      const int c = cb + sub + per * u;
      x[u] = c < C ? xin[c * FS + jr] : make_float2(0.f, 0.f);
    }
    lane_ifft(x, tw, F, jl, lane);
#pragma unroll
    for (int u = 0; u < kIlp; ++u) {
      const int c = cb + sub + per * u;
      if (c < C && m >= 0) xo[m * C + c] = x[u];
    }
  }
  __syncthreads();
  float2* dst = out + size_t(o) * B * inner;
  for (int e = threadIdx.x; e < B * C; e += blockDim.x) {
    const int mm = e / C, c = e - mm * C;
    if (c0 + c < inner) dst[size_t(mm) * inner + c0 + c] = xo[e];
  }
}

// Middle inverse pass: in [outer][F][inner] -> out [outer][B][inner]
__global__ void __launch_bounds__(256) k_inv_mid(const float2* __restrict__ in,
                                                 float2* __restrict__ out, PassGeom g,
                                                 int F, int inner, int B) {
  __shared__ float2 sa[2 * 256 * 2];
  float2* a = sa;
  float2* b = sa + 2 * 256;
  int ln, bt;
  map_thread<false>(g, &ln, &bt);
  const int line = blockIdx.x * g.lpb + ln;
  const bool active = line < g.nlines;
  const int outer = active ? line / inner : 0, in_i = active ? line % inner : 0;
  if (active)
    for (int j = bt; j < g.L; j += g.thr)
      a[ln * g.L + j] = in[(size_t(outer) * F + j) * inner + in_i];
  __syncthreads();
  float2* r = lds_fft(a, b, g.L, ln, bt, active, +1.f);
  if (active)
    for (int m = bt; m < B; m += g.thr)
      out[(size_t(outer) * B + m) * inner + in_i] = r[ln * g.L + lag_position(m, B, F)];
}

// Last inverse pass along x (contiguous lines): in [lines][F] -> R [lines][B]
// scaled by 1 / (F0 F1 F2).
__global__ void __launch_bounds__(256) k_inv_x(const float2* __restrict__ in,
                                               float2* __restrict__ out, PassGeom g, int F,
                                               int B, float scale) {
  __shared__ float2 sa[2 * 256 * 2];
  float2* a = sa;
  float2* b = sa + 2 * 256;
  int ln, bt;
  map_thread<true>(g, &ln, &bt);
  const int line = blockIdx.x * g.lpb + ln;
  const bool active = line < g.nlines && ln < g.lpb;
  if (active)
    for (int j = bt; j < g.L; j += g.thr) a[ln * g.L + j] = in[size_t(line) * F + j];
  __syncthreads();
  float2* r = lds_fft(a, b, g.L, ln, bt, active, +1.f);
  if (active)
    for (int m = bt; m < B; m += g.thr)
      out[size_t(line) * B + m] = cscale(r[ln * g.L + lag_position(m, B, F)], scale);
}

// ---------------------------------------------------------------- gather

// gram[(p,i),(q,j)] = R_pq[n_i - n_j] for row <= col; the lower triangle is
// the conjugate of the upper one and the diagonal is real.
__global__ void __launch_bounds__(256) k_gather(const float2* __restrict__ R,
                                                const int4* __restrict__ sup,
                                                float2* __restrict__ gram, int Q, int L,
                                                int B0, int B1, int B2, int nlag) {
  const int n = Q * L;
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (c >= n) return;
  // (coil, support point) of the row once per workgroup; of the column by a
  // float reciprocal with a one-step correction (exact: n <= 32 x 4096 = 2^17,
  // far below where the estimate could be off by more than one)
  const int pr = r / L, ir = r - pr * L;
  int pc = __float2int_rz(float(c) * (1.0f / float(L)));
  int ic = c - pc * L;
  if (ic < 0) {
    --pc;
    ic += L;
  } else if (ic >= L) {
    ++pc;
    ic -= L;
  }
  const bool up = r <= c;
  const int p = up ? pr : pc, i = up ? ir : ic, q = up ? pc : pr, j = up ? ic : ir;
  const int4 ni = sup[i], nj = sup[j];
  const int dz = ni.x - nj.x + (B0 - 1) / 2;
  const int dy = ni.y - nj.y + (B1 - 1) / 2;
  const int dx = ni.z - nj.z + (B2 - 1) / 2;
  const int pair = p * Q - p * (p - 1) / 2 + (q - p);
  float2 v = R[size_t(pair) * nlag + (dz * B1 + dy) * B2 + dx];
  if (r > c) v = cconj(v);
  if (r == c) v.y = 0.f;
  gram[size_t(r) * n + c] = v;
}

static unsigned blocks_for(const PassGeom& g) { return ceil_div(g.nlines, g.lpb); }

// ---------------------------------------------------------------- masked Gram

// Rows of C_valid (Eq. 5 with no implicit zeros): row v is the point n of
// the box [-floor(A/2) + tau, A - 1 - floor(A/2) - tau] per dimension
// (lexicographic, z slowest), column q |Lambda| + i holds s_q[n - n_i].
__global__ void k_cvalid(const float2* __restrict__ acs, const int4* __restrict__ sup,
                         float2* __restrict__ C, int Q, int L, int A0, int A1, int A2, int tz,
                         int tau, long long Pv, unsigned* status) {
  const int n = Q * L;
  const long long idx = blockIdx.x * 256LL + threadIdx.x;
  if (idx >= Pv * n) return;
  const long long v = idx / n;
  const int col = int(idx - v * n);
  const int q = col / L, i = col - q * L;
  const int V1 = A1 - 2 * tau, V2 = A2 - 2 * tau;
  const int vz = int(v / (1LL * V1 * V2)), vr = int(v - 1LL * vz * V1 * V2);
  const int vy = vr / V2, vx = vr - vy * V2;
  // array index of s_q[n - n_i]: n has array index (vz + tz, vy + tau, vx + tau)
  const int4 ni = sup[i];
  const int az = vz + tz - ni.x, ay = vy + tau - ni.y, ax = vx + tau - ni.z;
  float2 s = acs[((size_t(q) * A0 + az) * A1 + ay) * A2 + ax];
  if (!isfinite(s.x) || !isfinite(s.y)) {
    atomicOr(status, PISCO_FLAG_NONFINITE);
    s = make_float2(0.f, 0.f);
  }
  C[idx] = s;
}

// gram = C^H C for C [Pv][n] row-major (FP32 products, FP32 sums).  One
// workgroup per 32 x 32 block of the upper triangle (block row <= block
// column), 256 threads with 2 x 2 complex entries each; rows of C staged in
// LDS 16 at a time.  The lower triangle is written as the conjugate of the
// upper one and the diagonal is real, as for the correlation Gram.
__global__ void __launch_bounds__(256) k_cherk_valid(const float2* __restrict__ C,
                                                     float2* __restrict__ gram, int n,
                                                     long long Pv) {
  const int bi = blockIdx.y, bj = blockIdx.x;
  if (bi > bj) return;
  __shared__ float2 ta[16][33], tb[16][33];
  const int t = threadIdx.x;
  const int tr = t / 16, tc = t % 16;  // entries (2 tr + a, 2 tc + b) of the block
  const int r0 = bi * 32, c0 = bj * 32;
  float2 acc[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) acc[a][b] = make_float2(0.f, 0.f);
  for (long long v0 = 0; v0 < Pv; v0 += 16) {
    for (int e = t; e < 16 * 32; e += 256) {
      const int rr = e / 32, cc = e % 32;
      const long long v = v0 + rr;
      const bool okv = v < Pv;
      ta[rr][cc] = okv && r0 + cc < n ? C[size_t(v) * n + r0 + cc] : make_float2(0.f, 0.f);
      tb[rr][cc] = okv && c0 + cc < n ? C[size_t(v) * n + c0 + cc] : make_float2(0.f, 0.f);
    }
    __syncthreads();
#pragma unroll 4
    for (int k = 0; k < 16; ++k) {
      const float2 x0 = ta[k][2 * tr], x1 = ta[k][2 * tr + 1];
      const float2 y0 = tb[k][2 * tc], y1 = tb[k][2 * tc + 1];
      const float2 xs[2] = {x0, x1}, ys[2] = {y0, y1};
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          // conj(x) y
          acc[a][b].x = fmaf(xs[a].x, ys[b].x, fmaf(xs[a].y, ys[b].y, acc[a][b].x));
          acc[a][b].y = fmaf(xs[a].x, ys[b].y, fmaf(-xs[a].y, ys[b].x, acc[a][b].y));
        }
    }
    __syncthreads();
  }
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) {
      const int r = r0 + 2 * tr + a, c = c0 + 2 * tc + b;
      if (r >= n || c >= n || r > c) continue;
      float2 v = acc[a][b];
      if (r == c) v.y = 0.f;
      gram[size_t(r) * n + c] = v;
      if (r != c) gram[size_t(c) * n + r] = cconj(v);
    }
}

static pisco_status_t run_gram_valid(Handle* h, const Plan& p, const Tables& t, const float2* acs,
                                     float2* gram, void* ws) {
  GramWs w;
  layout_gram(p, ws, &w);
  const int n = p.n;
  const long long total = p.Pvalid * n;
  PISCO_KERNEL(h, k_cvalid, dim3(ceil_div(total, 256)), dim3(256), 0, acs, t.sup, w.C, p.Q, p.L,
               p.acs[0], p.acs[1], p.acs[2], p.D == 3 ? p.tau : 0, p.tau, p.Pvalid,
               h->status_dev);
  const unsigned nb = ceil_div(n, 32);
  PISCO_KERNEL(h, k_cherk_valid, dim3(nb, nb), dim3(256), 0, w.C, gram, n, p.Pvalid);
  return PISCO_OK;
}

// First inverse pass: S [Q][F][inner] -> out [P][B][inner].  The column-block
// kernel where F <= 64 and C >= 1 columns of all Q spectra fit in 64 KB of
// LDS (C a power of two up to 8); the line-per-pair kernel otherwise.
static pisco_status_t inv_first(Handle* h, const float2* S, float2* out, int Q, int F,
                                int inner, int B) {
  int logF = 0;
  while ((1 << logF) < F) ++logF;
  int C = 8;
  while (C > 0 && size_t(Q) * F * C * sizeof(float2) > 65536) C >>= 1;
  if ((1 << logF) == F && F <= 64 && C >= 1) {
    // few column blocks (2D): the channel pairs split over workgroups too,
    // about two workgroups per CU, at least eight pairs (one per wave) each
    const int P = Q * (Q + 1) / 2;
    const long long cblocks = ceil_div(inner, C);
    long long groups = (2LL * h->num_cu + cblocks - 1) / cblocks;
    const long long gmax = (P + 7) / 8;
    groups = groups < 1 ? 1 : (groups > gmax ? gmax : groups);
    PISCO_KERNEL(h, k_inv_first_cols, dim3(unsigned(cblocks), unsigned(groups)), dim3(512),
                 size_t(Q) * F * C * sizeof(float2), S, out, Q, F, logF, inner, B, C);
    return PISCO_OK;
  }
  const int P = Q * (Q + 1) / 2;
  PassGeom g = geom(F, 1LL * P * inner);
  PISCO_KERNEL(h, k_inv_first, dim3(blocks_for(g)), dim3(256), 0, S, out, g, Q, F, inner, B);
  return PISCO_OK;
}

pisco_status_t run_gram(Handle* h, const Plan& p, const Tables& t, const float2* acs,
                        float2* gram, void* ws, float2* lags_out) {
  if (p.rows == PISCO_ROWS_VALID) return run_gram_valid(h, p, t, acs, gram, ws);
  GramWs w;
  layout_gram(p, ws, &w);
  pisco_status_t st;
  const int Q = p.Q, P = p.P;
  const int A0 = p.acs[0], A1 = p.acs[1], A2 = p.acs[2];
  const int F0 = p.F[0], F1 = p.F[1], F2 = p.F[2];
  const int B0 = p.B[0], B1 = p.B[1], B2 = p.B[2];
  const int4* support = t.sup;

  // forward: x, y, (z)
  float2* S1 = w.S;                                   // [Q][A0][A1][F2]
  float2* S2 = w.S + size_t(Q) * F0 * F1 * F2;        // second half
  PassGeom gx = geom(F2, 1LL * Q * A0 * A1);
  PISCO_KERNEL(h, k_fwd_x, dim3(blocks_for(gx)), dim3(256), 0, acs, S1, gx, A2, F2, h->status_dev);
  PassGeom gy = geom(F1, 1LL * Q * A0 * F2);
  // 2D: S = S2 is [Q][1][F1][F2];  3D: S2 is [Q][A0][F1][F2]
  PISCO_KERNEL(h, k_fwd_mid, dim3(blocks_for(gy)), dim3(256), 0, S1, S2, gy, A1, F1, F2);
  const float2* Sfull = S2;
  if (p.D == 3) {
    PassGeom gz = geom(F0, 1LL * Q * F1 * F2);
    PISCO_KERNEL(h, k_fwd_mid, dim3(blocks_for(gz)), dim3(256), 0, S2, S1, gz, A0, F0, F1 * F2);
    Sfull = S1;  // [Q][F0][F1][F2]
  }

  // inverse per pair: (z), y, x
  const float scale = 1.0f / float(p.nF);
  if (p.D == 3) {
    if ((st = inv_first(h, Sfull, w.T1, Q, F0, F1 * F2, B0))) return st;
    PassGeom iy = geom(F1, 1LL * P * B0 * F2);
    if (F1 <= 64 && (F1 & (F1 - 1)) == 0) {
      int logF = 0;
      while ((1 << logF) < F1) ++logF;
      const int C = F2 < 64 ? F2 : 64;
      PISCO_KERNEL(h, k_inv_mid_cols, dim3(unsigned(1LL * P * B0 * ceil_div(F2, C))), dim3(512),
                   0, w.T1, w.T2, F1, logF, F2, B1, C);
    } else {
      PISCO_KERNEL(h, k_inv_mid, dim3(blocks_for(iy)), dim3(256), 0, w.T1, w.T2, iy, F1, F2, B1);
    }
  } else {
    if ((st = inv_first(h, Sfull, w.T2, Q, F1, F2, B1))) return st;
  }
  PassGeom ix = geom(F2, 1LL * P * B0 * B1);
  float2* R = lags_out ? lags_out : w.R;
  PISCO_KERNEL(h, k_inv_x, dim3(blocks_for(ix)), dim3(256), 0, w.T2, R, ix, F2, B2, scale);
  if (lags_out) return PISCO_OK;  // the caller multiplies through the lags

  dim3 gg(ceil_div(p.n, 256), p.n);
  PISCO_KERNEL(h, k_gather, gg, dim3(256), 0, w.R, support, gram, Q, p.L, B0, B1, B2, p.nlag);
  return PISCO_OK;
}

size_t gram_static_bytes(const Plan& p) {
  return ((layout_gram(p, nullptr, nullptr) + 255) & ~size_t(255)) +
         layout_tables(p, kTabSupport, nullptr, nullptr);
}

pisco_status_t run_gram_static(Handle* h, const Plan& p, const float2* acs, float2* gram) {
  const size_t need = gram_static_bytes(p);
  if (need > kGramScratchBytes) {
    h->last_error = "pisco_gram_static: problem needs " + std::to_string(need) +
                    " bytes of scratch, more than the library's " +
                    std::to_string(kGramScratchBytes);
    return PISCO_ERR_UNSUPPORTED;
  }
  void* base = nullptr;
  pisco_status_t st = gram_scratch_address(h, &base);
  if (st) return st;
  char* c = static_cast<char*>(base);
  const size_t off = (layout_gram(p, nullptr, nullptr) + 255) & ~size_t(255);
  Tables t;
  layout_tables(p, kTabSupport, c + off, &t);
  if ((st = build_tables(h, p, kTabSupport, t))) return st;
  return run_gram(h, p, t, acs, gram, c);
}

}  // namespace pisco
