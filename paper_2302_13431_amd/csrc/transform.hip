// Separable small-matrix transforms along one axis of a batched 3D array, and
// the device-side builders of the matrices they apply (DFT, apodized DFT,
// periodic sinc interpolation).  Every multi-dimensional transform of the path
// outside the Gram FFTs (filter spectra, lag kernel, G(x) evaluation, the
// apodized low-resolution image and the interpolation) is a product of such
// one-axis passes.
#include <cmath>

#include "common.hpp"

namespace pisco {

// out[outer][o][inner] = sum_i M[o][i] in[outer][i][inner]   (inner > 1)
// One thread per (outer, inner) column; 8 outputs per pass over the inputs.
__global__ void __launch_bounds__(256) k_axis_mid(const float2* __restrict__ in,
                                                  float2* __restrict__ out,
                                                  const float2* __restrict__ M,
                                                  long long outer, int nin, int nout,
                                                  int inner) {
  const long long col = blockIdx.x * 256LL + threadIdx.x;
  if (col >= outer * inner) return;
  const long long ou = col / inner;
  const int ii = int(col - ou * inner);
  const float2* src = in + size_t(ou) * nin * inner + ii;
  float2* dst = out + size_t(ou) * nout * inner + ii;
  for (int o0 = 0; o0 < nout; o0 += 8) {
    float2 acc[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) acc[k] = make_float2(0.f, 0.f);
    const int cnt = nout - o0 < 8 ? nout - o0 : 8;
    for (int i = 0; i < nin; ++i) {
      const float2 x = src[size_t(i) * inner];
#pragma unroll
      for (int k = 0; k < 8; ++k)
        if (k < cnt) {
          const float2 m = M[size_t(o0 + k) * nin + i];
          acc[k].x = fmaf(m.x, x.x, fmaf(-m.y, x.y, acc[k].x));
          acc[k].y = fmaf(m.x, x.y, fmaf(m.y, x.x, acc[k].y));
        }
    }
#pragma unroll
    for (int k = 0; k < 8; ++k)
      if (k < cnt) dst[size_t(o0 + k) * inner] = acc[k];
  }
}

// out[line][o] = sum_i M[o][i] in[line][i]   (contiguous lines)
// A block stages 16 lines in LDS; thread (line, o) computes one output.
__global__ void __launch_bounds__(256) k_axis_last(const float2* __restrict__ in,
                                                   float2* __restrict__ out,
                                                   const float2* __restrict__ M,
                                                   long long lines, int nin, int nout) {
  extern __shared__ float2 sl[];  // [16][nin]
  const long long l0 = blockIdx.x * 16LL;
  const int nl = lines - l0 < 16 ? int(lines - l0) : 16;
  for (int e = threadIdx.x; e < nl * nin; e += 256) sl[e] = in[size_t(l0) * nin + e];
  __syncthreads();
  for (int e = threadIdx.x; e < nl * nout; e += 256) {
    const int ln = e / nout, o = e - ln * nout;
    const float2* x = sl + ln * nin;
    const float2* m = M + size_t(o) * nin;
    float ar = 0.f, ai = 0.f;
    for (int i = 0; i < nin; ++i) {
      const float2 mv = m[i], xv = x[i];
      ar = fmaf(mv.x, xv.x, fmaf(-mv.y, xv.y, ar));
      ai = fmaf(mv.x, xv.y, fmaf(mv.y, xv.x, ai));
    }
    out[size_t(l0 + ln) * nout + o] = make_float2(ar, ai);
  }
}

pisco_status_t axis_transform(hipStream_t s, const float2* in, float2* out,
                              const int shape_in[4], int axis, int nout, const float2* M) {
  long long outer = shape_in[0];
  for (int d = 1; d < axis; ++d) outer *= shape_in[d];
  long long inner = 1;
  for (int d = axis + 1; d < 4; ++d) inner *= shape_in[d];
  const int nin = shape_in[axis];
  if (inner == 1) {
    const size_t lds = size_t(16) * nin * sizeof(float2);
    if (lds > 64 * 1024) return PISCO_ERR_UNSUPPORTED;
    hipLaunchKernelGGL(k_axis_last, dim3(ceil_div(outer, 16)), dim3(256), lds, s, in, out, M,
                       outer, nin, nout);
  } else {
    hipLaunchKernelGGL(k_axis_mid, dim3(ceil_div(outer * inner, 256)), dim3(256), 0, s, in,
                       out, M, outer, nin, nout, int(inner));
  }
  return hipGetLastError() == hipSuccess ? PISCO_OK : PISCO_ERR_HIP;
}

// ------------------------------------------------------------------ matrix builders

// M[o][i] = scale * w(i) * exp(i * sign * 2 pi * (i - ci) * (o - co) / period)
// with w(i) = exp(-(i - ci)^2 / (2 sigma^2)) when sigma > 0, else 1.
__global__ void k_build_dft(float2* M, int nout, int nin, int co, int ci, double period,
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
  M[idx] = make_float2(float(w * cs), float(w * sn));
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

pisco_status_t build_dft(hipStream_t s, float2* M, int nout, int nin, int co, int ci,
                         double period, double sign, double scale, double sigma) {
  hipLaunchKernelGGL(k_build_dft, dim3(ceil_div(nout * nin, 256)), dim3(256), 0, s, M, nout,
                     nin, co, ci, period, sign, scale, sigma);
  return hipGetLastError() == hipSuccess ? PISCO_OK : PISCO_ERR_HIP;
}

pisco_status_t build_sinc(hipStream_t s, float2* M, int nout, int nin) {
  hipLaunchKernelGGL(k_build_sinc, dim3(ceil_div(nout * nin, 256)), dim3(256), 0, s, M, nout,
                     nin);
  return hipGetLastError() == hipSuccess ? PISCO_OK : PISCO_ERR_HIP;
}

}  // namespace pisco
