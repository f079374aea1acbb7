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

template <class TI, class TO>
static pisco_status_t axis_impl(Handle* h, const TI* in, TO* out, const int shape_in[4],
                                int axis, int nout, const TO* M) {
  long long outer = shape_in[0];
  for (int d = 1; d < axis; ++d) outer *= shape_in[d];
  long long inner = 1;
  for (int d = axis + 1; d < 4; ++d) inner *= shape_in[d];
  const int nin = shape_in[axis];
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
                              int axis, int nout, const float2* M) {
  return axis_impl<float2, float2>(h, in, out, shape_in, axis, nout, M);
}

pisco_status_t axis_transform64(Handle* h, const float2* in, double2* out,
                                const int shape_in[4], int axis, int nout, const double2* M) {
  return axis_impl<float2, double2>(h, in, out, shape_in, axis, nout, M);
}

pisco_status_t axis_transform64(Handle* h, const double2* in, double2* out,
                                const int shape_in[4], int axis, int nout, const double2* M) {
  return axis_impl<double2, double2>(h, in, out, shape_in, axis, nout, M);
}

// ------------------------------------------------------------------ matrix builders

// M[o][i] = scale * w(i) * exp(i * sign * 2 pi * (i - ci) * (o - co) / period)
// with w(i) = exp(-(i - ci)^2 / (2 sigma^2)) when sigma > 0, else 1.
template <class TM>
__global__ void k_build_dft(TM* M, int nout, int nin, int co, int ci, double period,
                            double sign, double scale, double sigma) {
  const int idx = blockIdx.x * 256 + threadIdx.x;
  if (idx >= nout * nin) return;
  const int o = idx / nin, i = idx - o * nin;
  const long long prod = 1LL * (i - ci) * (o - co);
  // reduce the phase exactly in integers before the trigonometric call
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
  M[idx] = TM{static_cast<decltype(TM{}.x)>(w * cs), static_cast<decltype(TM{}.x)>(w * sn)};
}

// Periodic sinc (Dirichlet) interpolation from n_in to n_out >= n_in centred
// samples: M[o][a] = (1/n_in) sum_k w_k exp(i 2 pi k (y_o - x_a)) over the
// centred band of n_in frequencies, the -n_in/2 term split in half onto
// +-n_in/2 when n_in is even and n_out > n_in.
__global__ void k_build_sinc(float2* M, int nout, int nin) {
  const int idx = blockIdx.x * 256 + threadIdx.x;
  if (idx >= nout * nin) return;
  const int o = idx / nin, a = idx - o * nin;
  const int kmin = -(nin / 2), kmax = (nin + 1) / 2 - 1;
  const bool split = (nin % 2 == 0) && nout > nin;
  const double y = double(o - nout / 2) / double(nout);
  const double x = double(a - nin / 2) / double(nin);
  double re = 0.0, im = 0.0;
  for (int k = kmin; k <= kmax; ++k) {
    double sn, cs;
    sincospi(2.0 * double(k) * (y - x), &sn, &cs);
    const double w = (split && k == kmin) ? 0.5 : 1.0;
    re += w * cs;
    im += w * sn;
  }
  if (split) {
    double sn, cs;
    sincospi(2.0 * double(nin / 2) * (y - x), &sn, &cs);
    re += 0.5 * cs;
    im += 0.5 * sn;
  }
  M[idx] = make_float2(float(re / nin), float(im / nin));
}

pisco_status_t build_dft(Handle* h, float2* M, int nout, int nin, int co, int ci,
                         double period, double sign, double scale, double sigma) {
  PISCO_KERNEL(h, k_build_dft<float2>, dim3(ceil_div(nout * nin, 256)), dim3(256), 0, M, nout,
               nin, co, ci, period, sign, scale, sigma);
  return PISCO_OK;
}

pisco_status_t build_dft(Handle* h, double2* M, int nout, int nin, int co, int ci,
                         double period, double sign, double scale, double sigma) {
  PISCO_KERNEL(h, k_build_dft<double2>, dim3(ceil_div(nout * nin, 256)), dim3(256), 0, M, nout,
               nin, co, ci, period, sign, scale, sigma);
  return PISCO_OK;
}

pisco_status_t build_sinc(Handle* h, float2* M, int nout, int nin) {
  PISCO_KERNEL(h, k_build_sinc, dim3(ceil_div(nout * nin, 256)), dim3(256), 0, M, nout, nin);
  return PISCO_OK;
}

namespace {
template <class T>
pisco_status_t dft_table_t(Handle* h, const T** M, const char* tag, int nout, int nin, int co,
                           int ci, double period, double sign, double scale, double sigma) {
  char key[192];
  std::snprintf(key, sizeof key, "%s %d %d %d %d %.17g %.17g %.17g %.17g", tag, nout, nin, co,
                ci, period, sign, scale, sigma);
  void* p = nullptr;
  pisco_status_t st = cached_table(h, key, sizeof(T) * size_t(nout) * nin, &p,
                                   [&](void* q) {
                                     return build_dft(h, static_cast<T*>(q), nout, nin, co, ci,
                                                      period, sign, scale, sigma);
                                   });
  *M = static_cast<const T*>(p);
  return st;
}
}  // namespace

pisco_status_t dft_table(Handle* h, const float2** M, int nout, int nin, int co, int ci,
                         double period, double sign, double scale, double sigma) {
  return dft_table_t(h, M, "dft32", nout, nin, co, ci, period, sign, scale, sigma);
}

pisco_status_t dft_table(Handle* h, const double2** M, int nout, int nin, int co, int ci,
                         double period, double sign, double scale, double sigma) {
  return dft_table_t(h, M, "dft64", nout, nin, co, ci, period, sign, scale, sigma);
}

pisco_status_t sinc_table(Handle* h, const float2** M, int nout, int nin) {
  char key[64];
  std::snprintf(key, sizeof key, "sinc %d %d", nout, nin);
  void* p = nullptr;
  pisco_status_t st = cached_table(h, key, sizeof(float2) * size_t(nout) * nin, &p,
                                   [&](void* q) {
                                     return build_sinc(h, static_cast<float2*>(q), nout, nin);
                                   });
  *M = static_cast<const float2*>(p);
  return st;
}

}  // namespace pisco
