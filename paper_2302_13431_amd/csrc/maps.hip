// Phase reference, periodic sinc interpolation and sum-of-squares
// normalisation (Sec. IV-D, Sec. V).
//
// alpha(x) cancels the phase of the coil combination m(x) = c(x)^H rho~(x) of
// a Gaussian-apodized low-resolution reconstruction rho~ of the calibration
// data (apodization exp(-k^2 / (2 (A/4)^2)) per dimension), so the phase of
// the maps becomes as smooth as the maps themselves and they can be
// interpolated.  rho~ and m are formed in FP64: |m| is small outside the
// object, where FP32 cancellation would otherwise decide the phase.  Interpolation is the periodic sinc of a zero-padded spectrum,
// applied as one small matrix per dimension; the last step divides every
// output voxel by its root-sum-of-squares over coils.
#include "common.hpp"

namespace pisco {

// m[v] = sum_q conj(c_q[v]) rho_q[v] in FP64; partial max of |m| per block.
// The phase reference divides by |m|, which is small outside the object, so
// the combination is formed in FP64 from the FP32 maps and the FP64 image.
__global__ void __launch_bounds__(256) k_phase_m(const float2* __restrict__ c,
                                                 const double2* __restrict__ rho,
                                                 double2* __restrict__ m,
                                                 double* __restrict__ pmax, int Q,
                                                 long long N) {
  __shared__ double red[256];
  const long long v = blockIdx.x * 256LL + threadIdx.x;
  double mag = 0.0;
  if (v < N) {
    // coils in batches of eight, each batch's loads in flight together
    constexpr int kB = 8;
    double2 acc = make_double2(0.0, 0.0);
    for (int q0 = 0; q0 < Q; q0 += kB) {
      float2 a[kB];
      double2 r[kB];
#pragma unroll
      for (int u = 0; u < kB; ++u) {
        const bool ok = q0 + u < Q;
        a[u] = ok ? c[size_t(q0 + u) * N + v] : make_float2(0.f, 0.f);
        r[u] = ok ? rho[size_t(q0 + u) * N + v] : make_double2(0.0, 0.0);
      }
#pragma unroll
      for (int u = 0; u < kB; ++u) {
        if (q0 + u >= Q) break;
        acc.x = fma(double(a[u].x), r[u].x, fma(double(a[u].y), r[u].y, acc.x));
        acc.y = fma(double(a[u].x), r[u].y, fma(-double(a[u].y), r[u].x, acc.y));
      }
    }
    m[v] = acc;
    mag = sqrt(zabs2(acc));
  }
  red[threadIdx.x] = mag;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + off]);
    __syncthreads();
  }
  if (threadIdx.x == 0) pmax[blockIdx.x] = red[0];
}

// cref = c * m/|m| where |m| > 1e-12 max|m|, else c
__global__ void __launch_bounds__(256) k_phase_apply(const float2* __restrict__ c,
                                                     const double2* __restrict__ m,
                                                     const double* __restrict__ pmax, int nblk,
                                                     float2* __restrict__ cref, int Q,
                                                     long long N) {
  __shared__ double gmax;
  if (threadIdx.x < 64) {  // the block maxima, read by one wave in parallel
    double g = 0.0;
    for (int i = threadIdx.x; i < nblk; i += 64) g = fmax(g, pmax[i]);
    for (int off = 32; off > 0; off >>= 1) g = fmax(g, __shfl_xor(g, off, 64));
    if (threadIdx.x == 0) gmax = g;
  }
  __syncthreads();
  const long long v = blockIdx.x * 256LL + threadIdx.x;
  if (v >= N) return;
  const double2 mv = m[v];
  const double mag = sqrt(zabs2(mv));
  double2 a = make_double2(1.0, 0.0);
  if (mag > 1e-12 * gmax && mag > 0.0) a = make_double2(mv.x / mag, mv.y / mag);
  constexpr int kB = 8;  // coils in batches, each batch's loads in flight together
  for (int q0 = 0; q0 < Q; q0 += kB) {
    float2 cv[kB];
#pragma unroll
    for (int u = 0; u < kB; ++u)
      cv[u] = q0 + u < Q ? c[size_t(q0 + u) * N + v] : make_float2(0.f, 0.f);
#pragma unroll
    for (int u = 0; u < kB; ++u)
      if (q0 + u < Q)
        cref[size_t(q0 + u) * N + v] = make_float2(float(cv[u].x * a.x - cv[u].y * a.y),
                                                   float(cv[u].x * a.y + cv[u].y * a.x));
  }
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
// The voxel's Q coil values are loaded once, all loads in flight together,
// and kept in registers for the scaling.
__global__ void __launch_bounds__(256) k_rss(float2* __restrict__ c, int Q, long long N) {
  const long long v = blockIdx.x * 256LL + threadIdx.x;
  if (v >= N) return;
  float2 x[kMaxQ];
#pragma unroll
  for (int q = 0; q < kMaxQ; ++q) x[q] = q < Q ? c[size_t(q) * N + v] : make_float2(0.f, 0.f);
  float s = 0.f;
#pragma unroll
  for (int q = 0; q < kMaxQ; ++q) s += cabs2(x[q]);
  if (!(s > 0.f)) return;
  const float inv = 1.f / sqrtf(s);
#pragma unroll
  for (int q = 0; q < kMaxQ; ++q)
    if (q < Q) c[size_t(q) * N + v] = cscale(x[q], inv);
}

pisco_status_t run_maps(Handle* h, const Plan& p, const Tables& t, int phase_rule,
                        const float2* acs, const float2* maps_lr, float2* maps_out, void* ws) {
  MapsWs w;
  layout_maps(p, ws, &w);
  const int Q = p.Q;
  const long long N = p.Nlr;
  pisco_status_t st;
  // apodized DFT (acs -> lr, FP64) and sinc (lr -> out) per dimension
  const double2* const* Ma = t.Ma;
  const float2* const* Ms = t.Ms;
  if (phase_rule == 0) {
    // rho~ = apodized low-res reconstruction in FP64: [Q][A0][A1][A2] -> [Q][lr]
    int sh[4] = {Q, p.acs[0], p.acs[1], p.acs[2]};
    if ((st = axis_transform64(h, acs, w.rtA, sh, 3, p.lr[2], Ma[2]))) return st;
    sh[3] = p.lr[2];
    if (p.D == 3) {
      if ((st = axis_transform64(h, w.rtA, w.rtB, sh, 2, p.lr[1], Ma[1]))) return st;
      sh[2] = p.lr[1];
      if ((st = axis_transform64(h, w.rtB, w.rho, sh, 1, p.lr[0], Ma[0]))) return st;
    } else {
      if ((st = axis_transform64(h, w.rtA, w.rho, sh, 2, p.lr[1], Ma[1]))) return st;
    }
    const unsigned nblk = ceil_div(N, 256);
    PISCO_KERNEL(h, k_phase_m, dim3(nblk), dim3(256), 0, maps_lr, w.rho, w.m, w.pmax, Q, N);
    PISCO_KERNEL(h, k_phase_apply, dim3(nblk), dim3(256), 0, maps_lr, w.m, w.pmax, int(nblk),
                 w.cref, Q, N);
  } else {
    PISCO_KERNEL(h, k_phase_coil, dim3(ceil_div(N, 256)), dim3(256), 0, maps_lr, w.cref, Q, N);
  }
  // interpolation [Q][lr0][lr1][lr2] -> [Q][out0][out1][out2], one axis at a
  // time in the order interp_order gives (x last); the x pass carries the
  // coil normalisation
  int sh[4] = {Q, p.lr[0], p.lr[1], p.lr[2]};
  int ord[3];
  const int n = interp_order(p, ord);
  const float2* cur = w.cref;
  for (int i = 0; i + 1 < n; ++i) {
    const int d = ord[i];
    float2* dst = i == 0 ? w.tmpA : w.tmpB;
    if ((st = axis_transform(h, cur, dst, sh, d + 1, p.out[d], Ms[d], true))) return st;
    sh[d + 1] = p.out[d];
    cur = dst;
  }
  const long long rows = 1LL * p.out[0] * p.out[1];
  st = interp_x_rss(h, cur, maps_out, Ms[2], Q, rows, p.lr[2], p.out[2]);
  if (st == PISCO_ERR_UNSUPPORTED) {
    if ((st = axis_transform(h, cur, maps_out, sh, 3, p.out[2], Ms[2], true))) return st;
    PISCO_KERNEL(h, k_rss, dim3(ceil_div(p.Nout, 256)), dim3(256), 0, maps_out, Q, p.Nout);
  } else if (st) {
    return st;
  }
  return PISCO_OK;
}

}  // namespace pisco
