// Support mask and ESPIRiT operator form (Sec. III-B to III-E).
//
// Support mask (optional last step of the naive algorithm, Sec. III-D):
// inside the image support H(x) has rank Q - 1 and lambda_min(G(x)), the
// square of its smallest singular value, is about zero; outside, H(x) has
// full rank and lambda_min is clearly positive.  The low-resolution map
// lambda_min / |Lambda| (in [0, 1]) is brought to the output grid by the
// same periodic sinc interpolation as the maps, here in FP64 so that the
// threshold decision is taken on values accurate to rounding, and a voxel is
// inside where the interpolated value is below the threshold.
//
// ESPIRiT operator (Eq. 20): B(x) = I - G(x) / |Lambda|, the operator whose
// eigenvector for eigenvalue one (the largest) is the map; written in the
// packed entry-major layout of G.
#include "common.hpp"

namespace pisco {

// t0[v] = lam[v] / bound as a complex FP64 value
__global__ void k_mask_load(const float* __restrict__ lam, double2* __restrict__ t0,
                            long long N, double inv_bound) {
  const long long v = blockIdx.x * 256LL + threadIdx.x;
  if (v < N) t0[v] = make_double2(double(lam[v]) * inv_bound, 0.0);
}

__global__ void k_mask_threshold(const double2* __restrict__ up, uint8_t* __restrict__ mask,
                                 long long N, double thresh) {
  const long long v = blockIdx.x * 256LL + threadIdx.x;
  if (v < N) mask[v] = up[v].x < thresh ? 1 : 0;
}

size_t layout_mask(const Plan& p, void* ws, double2** t0, double2** t1, double2** t2) {
  Carver c(ws);
  const size_t a = size_t(p.lr[0]) * p.lr[1] * p.out[2];
  const size_t b = size_t(p.lr[0]) * p.out[1] * p.out[2];
  const size_t n = size_t(p.Nout) > a ? size_t(p.Nout) : a;
  double2* x0 = c.take<double2>(p.Nlr);
  double2* x1 = c.take<double2>(n);
  double2* x2 = c.take<double2>(b);
  if (t0) *t0 = x0;
  if (t1) *t1 = x1;
  if (t2) *t2 = x2;
  return c.used + 256;
}

pisco_status_t run_support_mask(Handle* h, const Plan& p, const Tables& t, const float* lam,
                                float bound, float thresh, uint8_t* mask, void* ws) {
  double2 *t0, *t1, *t2;
  layout_mask(p, ws, &t0, &t1, &t2);
  PISCO_KERNEL(h, k_mask_load, dim3(ceil_div(p.Nlr, 256)), dim3(256), 0, lam, t0, p.Nlr,
               1.0 / double(bound));
  // [1][lr0][lr1][lr2] -> x -> y -> (z)
  int sh[4] = {1, p.lr[0], p.lr[1], p.lr[2]};
  pisco_status_t st;
  if ((st = axis_transform64(h, t0, t1, sh, 3, p.out[2], t.Ms64[2]))) return st;
  sh[3] = p.out[2];
  const double2* up = nullptr;
  if (p.D == 3) {
    if ((st = axis_transform64(h, t1, t2, sh, 2, p.out[1], t.Ms64[1]))) return st;
    sh[2] = p.out[1];
    if ((st = axis_transform64(h, t2, t1, sh, 1, p.out[0], t.Ms64[0]))) return st;
    up = t1;
  } else {
    if ((st = axis_transform64(h, t1, t2, sh, 2, p.out[1], t.Ms64[1]))) return st;
    up = t2;
  }
  PISCO_KERNEL(h, k_mask_threshold, dim3(ceil_div(p.Nout, 256)), dim3(256), 0, up, mask, p.Nout,
               double(thresh));
  return PISCO_OK;
}

// B = delta - G / bound on the packed planes [Q(Q+1)/2][N]; diagonal real
__global__ void k_espirit_op(const float2* __restrict__ G, float2* __restrict__ B, int Q,
                             long long N, float inv_bound) {
  const long long idx = blockIdx.x * 256LL + threadIdx.x;
  const int P = Q * (Q + 1) / 2;
  if (idx >= 1LL * P * N) return;
  const int pair = int(idx / N);
  int p = 0, base = 0;
  while (pair >= base + (Q - p)) {
    base += Q - p;
    ++p;
  }
  const bool diag = pair == base;
  const float2 g = G[idx];
  B[idx] = diag ? make_float2(1.f - g.x * inv_bound, 0.f)
                : make_float2(-g.x * inv_bound, -g.y * inv_bound);
}

pisco_status_t run_espirit_operator(Handle* h, int Q, long long N, float bound,
                                    const float2* G, float2* B) {
  if (N <= 0) return PISCO_OK;
  const long long total = 1LL * Q * (Q + 1) / 2 * N;
  PISCO_KERNEL(h, k_espirit_op, dim3(ceil_div(total, 256)), dim3(256), 0, G, B, Q, N,
               1.f / bound);
  return PISCO_OK;
}

}  // namespace pisco
