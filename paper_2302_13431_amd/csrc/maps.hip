// Phase reference, periodic sinc interpolation and sum-of-squares
// normalisation (Sec. IV-D, Sec. V).
//
// alpha(x) cancels the phase of the coil combination m(x) = c(x)^H rho~(x) of
// a Gaussian-apodized low-resolution reconstruction rho~ of the calibration
// data (apodization exp(-k^2 / (2 (A/4)^2)) per dimension), so the phase of
// the maps becomes as smooth as the maps themselves and they can be
// interpolated.  Interpolation is the periodic sinc of a zero-padded spectrum,
// applied as one small matrix per dimension; the last step divides every
// output voxel by its root-sum-of-squares over coils.
#include "common.hpp"

namespace pisco {

// m[v] = sum_q conj(c_q[v]) rho_q[v]; partial max of |m| per block
__global__ void __launch_bounds__(256) k_phase_m(const float2* __restrict__ c,
                                                 const float2* __restrict__ rho,
                                                 float2* __restrict__ m,
                                                 float* __restrict__ pmax, int Q,
                                                 long long N) {
  __shared__ float red[256];
  const long long v = blockIdx.x * 256LL + threadIdx.x;
  float mag = 0.f;
  if (v < N) {
    float2 acc = make_float2(0.f, 0.f);
    for (int q = 0; q < Q; ++q) {
      const float2 a = c[size_t(q) * N + v], r = rho[size_t(q) * N + v];
      acc.x = fmaf(a.x, r.x, fmaf(a.y, r.y, acc.x));
      acc.y = fmaf(a.x, r.y, fmaf(-a.y, r.x, acc.y));
    }
    m[v] = acc;
    mag = sqrtf(cabs2(acc));
  }
  red[threadIdx.x] = mag;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + off]);
    __syncthreads();
  }
  if (threadIdx.x == 0) pmax[blockIdx.x] = red[0];
}

// cref = c * m/|m| where |m| > 1e-12 max|m|, else c
__global__ void __launch_bounds__(256) k_phase_apply(const float2* __restrict__ c,
                                                     const float2* __restrict__ m,
                                                     const float* __restrict__ pmax, int nblk,
                                                     float2* __restrict__ cref, int Q,
                                                     long long N) {
  __shared__ float gmax;
  if (threadIdx.x == 0) {
    float g = 0.f;
    for (int i = 0; i < nblk; ++i) g = fmaxf(g, pmax[i]);
    gmax = g;
  }
  __syncthreads();
  const long long v = blockIdx.x * 256LL + threadIdx.x;
  if (v >= N) return;
  const float2 mv = m[v];
  const float mag = sqrtf(cabs2(mv));
  float2 a = make_float2(1.f, 0.f);
  if (mag > 1e-12f * gmax && mag > 0.f) a = make_float2(mv.x / mag, mv.y / mag);
  for (int q = 0; q < Q; ++q) cref[size_t(q) * N + v] = cmul(c[size_t(q) * N + v], a);
}

// cref = c * conj(c_0)/|c_0|  (phase referenced to channel 0)
__global__ void __launch_bounds__(256) k_phase_coil(const float2* __restrict__ c,
                                                    float2* __restrict__ cref, int Q,
                                                    long long N) {
  const long long v = blockIdx.x * 256LL + threadIdx.x;
  if (v >= N) return;
  const float2 r = c[v];
  const float mag = sqrtf(cabs2(r));
  const float2 a = mag > 0.f ? make_float2(r.x / mag, -r.y / mag) : make_float2(1.f, 0.f);
  for (int q = 0; q < Q; ++q) cref[size_t(q) * N + v] = cmul(c[size_t(q) * N + v], a);
}

// c[:, v] /= ||c[:, v]||_2 (zero stays zero)
__global__ void __launch_bounds__(256) k_rss(float2* __restrict__ c, int Q, long long N) {
  const long long v = blockIdx.x * 256LL + threadIdx.x;
  if (v >= N) return;
  float s = 0.f;
  for (int q = 0; q < Q; ++q) s += cabs2(c[size_t(q) * N + v]);
  if (!(s > 0.f)) return;
  const float inv = 1.f / sqrtf(s);
  for (int q = 0; q < Q; ++q) c[size_t(q) * N + v] = cscale(c[size_t(q) * N + v], inv);
}

pisco_status_t run_maps(Handle* h, const Plan& p, int phase_rule, const float2* acs,
                        const float2* maps_lr, float2* maps_out, void* ws) {
  MapsWs w;
  layout_maps(p, ws, &w);
  hipStream_t s = h->stream;
  const int Q = p.Q;
  const long long N = p.Nlr;
  pisco_status_t st;
  const int first = p.D == 3 ? 0 : 1;
  // matrices: apodized DFT (acs -> lr) and sinc (lr -> out) per dimension
  float2* m = w.Mx;
  float2* Ma[3];
  float2* Ms[3];
  for (int d = 0; d < 3; ++d) {
    Ma[d] = m;
    m += size_t(p.lr[d]) * p.acs[d];
    Ms[d] = m;
    m += size_t(p.out[d]) * p.lr[d];
    if (d < first) continue;
    const int A = p.acs[d], n = p.lr[d];
    if ((st = build_dft(s, Ma[d], n, A, n / 2, A / 2, n, +1.0, 1.0, A / 4.0))) return st;
    if ((st = build_sinc(s, Ms[d], p.out[d], n))) return st;
  }
  if (phase_rule == 0) {
    // rho~ = apodized low-res reconstruction: [Q][A0][A1][A2] -> [Q][lr]
    int sh[4] = {Q, p.acs[0], p.acs[1], p.acs[2]};
    if ((st = axis_transform(s, acs, w.tmpA, sh, 3, p.lr[2], Ma[2]))) return st;
    sh[3] = p.lr[2];
    if (p.D == 3) {
      if ((st = axis_transform(s, w.tmpA, w.tmpB, sh, 2, p.lr[1], Ma[1]))) return st;
      sh[2] = p.lr[1];
      if ((st = axis_transform(s, w.tmpB, w.rho, sh, 1, p.lr[0], Ma[0]))) return st;
    } else {
      if ((st = axis_transform(s, w.tmpA, w.rho, sh, 2, p.lr[1], Ma[1]))) return st;
    }
    const unsigned nblk = ceil_div(N, 256);
    float2* mbuf = w.tmpA;                              // [N]
    float* pmax = reinterpret_cast<float*>(w.tmpB);     // [nblk]
    hipLaunchKernelGGL(k_phase_m, dim3(nblk), dim3(256), 0, s, maps_lr, w.rho, mbuf, pmax, Q,
                       N);
    PISCO_LAUNCH_CHECK(h, "maps phase m");
    hipLaunchKernelGGL(k_phase_apply, dim3(nblk), dim3(256), 0, s, maps_lr, mbuf, pmax,
                       int(nblk), w.cref, Q, N);
    PISCO_LAUNCH_CHECK(h, "maps phase apply");
  } else {
    hipLaunchKernelGGL(k_phase_coil, dim3(ceil_div(N, 256)), dim3(256), 0, s, maps_lr, w.cref,
                       Q, N);
    PISCO_LAUNCH_CHECK(h, "maps phase coil");
  }
  // interpolation: [Q][lr0][lr1][lr2] -> x -> y -> (z) -> maps_out
  int sh[4] = {Q, p.lr[0], p.lr[1], p.lr[2]};
  if ((st = axis_transform(s, w.cref, w.tmpA, sh, 3, p.out[2], Ms[2]))) return st;
  sh[3] = p.out[2];
  if (p.D == 3) {
    if ((st = axis_transform(s, w.tmpA, w.tmpB, sh, 2, p.out[1], Ms[1]))) return st;
    sh[2] = p.out[1];
    if ((st = axis_transform(s, w.tmpB, maps_out, sh, 1, p.out[0], Ms[0]))) return st;
  } else {
    if ((st = axis_transform(s, w.tmpA, maps_out, sh, 2, p.out[1], Ms[1]))) return st;
  }
  hipLaunchKernelGGL(k_rss, dim3(ceil_div(p.Nout, 256)), dim3(256), 0, s, maps_out, Q, p.Nout);
  PISCO_LAUNCH_CHECK(h, "maps rss");
  return PISCO_OK;
}

}  // namespace pisco
