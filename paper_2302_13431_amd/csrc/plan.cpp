// Host-side problem planning: support enumeration, derived sizes and the
// workspace layout of every stage.
#include <cmath>
#include <cstdio>

#include "common.hpp"

namespace pisco {

int enumerate_support(int D, float radius, int shape, int32_t* offsets, int cap) {
  // Lambda = { n in Z^D : ||n||_2 <= radius } (Sec. IV-B) or the box
  // ||n||_inf <= floor(radius) (Sec. III-C), lexicographic order with z
  // slowest and x fastest.  For D = 2 the z offset is 0.
  const int t = static_cast<int>(std::floor(radius));
  const double r2 = double(radius) * double(radius);
  const int zlo = (D == 3) ? -t : 0, zhi = (D == 3) ? t : 0;
  int count = 0;
  for (int z = zlo; z <= zhi; ++z)
    for (int y = -t; y <= t; ++y)
      for (int x = -t; x <= t; ++x) {
        if (shape == PISCO_SHAPE_ELLIPSOID && double(z) * z + double(y) * y + double(x) * x > r2)
          continue;
        if (offsets && count < cap) {
          offsets[3 * count + 0] = z;
          offsets[3 * count + 1] = y;
          offsets[3 * count + 2] = x;
        }
        ++count;
      }
  return count;
}

static int next_pow2(int v) {
  int p = 1;
  while (p < v) p <<= 1;
  return p;
}

pisco_status_t make_plan(const pisco_problem_t* prob, Plan* p, std::string* err) {
  auto fail = [&](const char* m) {
    if (err) *err = m;
    return PISCO_ERR_ARG;
  };
  if (!prob) return fail("problem is NULL");
  if (prob->D != 2 && prob->D != 3) return fail("D must be 2 or 3");
  if (prob->Q < 2 || prob->Q > kMaxQ) return fail("Q must be in [2, 32]");
  if (!(prob->radius >= 1.0f) || prob->radius > 12.0f)
    return fail("radius must be in [1, 12]");
  if (!(prob->thresh > 0.0f) || prob->thresh >= 1.0f)
    return fail("thresh must be in (0, 1)");
  if (prob->shape != PISCO_SHAPE_ELLIPSOID && prob->shape != PISCO_SHAPE_RECTANGLE)
    return fail("unknown support shape");
  if (prob->gram_rows != PISCO_ROWS_ALL && prob->gram_rows != PISCO_ROWS_VALID)
    return fail("unknown gram_rows");
  p->shape = prob->shape;
  p->rows = prob->gram_rows;
  p->D = prob->D;
  p->Q = prob->Q;
  p->radius = prob->radius;
  p->tau = static_cast<int>(std::floor(prob->radius));
  p->thresh = prob->thresh;
  const int first = (p->D == 3) ? 0 : 1;
  for (int d = 0; d < 3; ++d) {
    const bool used = d >= first;
    p->acs[d] = used ? prob->acs[d] : 1;
    p->lr[d] = used ? prob->grid_lr[d] : 1;
    p->out[d] = used ? prob->grid_out[d] : 1;
    if (!used && (prob->acs[d] > 1 || prob->grid_lr[d] > 1 || prob->grid_out[d] > 1))
      return fail("z extents must be 1 when D = 2");
    if (used) {
      if (p->acs[d] <= 2 * p->tau) return fail("ACS extent must exceed 2 * radius");
      if (p->lr[d] < 1 || p->out[d] < p->lr[d])
        return fail("need 1 <= grid_lr <= grid_out in every dimension");
    }
    p->B[d] = used ? 4 * p->tau + 1 : 1;
    p->F[d] = used ? next_pow2(p->acs[d] + 2 * p->tau) : 1;
    p->K[d] = p->B[d];
    if (p->F[d] > 256) return fail("ACS + 2 * radius must be <= 256 per dimension");
    if (p->lr[d] > 1024 || p->out[d] > 4096) return fail("grid too large");
  }
  p->L = enumerate_support(p->D, p->radius, p->shape, nullptr, 0);
  p->Pvalid = 1;
  for (int d = first; d < 3; ++d) p->Pvalid *= p->acs[d] - 2 * p->tau;
  if (p->L > kMaxSupport) return fail("support too large");
  p->n = p->Q * p->L;
  p->P = p->Q * (p->Q + 1) / 2;
  p->nlag = p->B[0] * p->B[1] * p->B[2];
  p->nF = p->F[0] * p->F[1] * p->F[2];
  p->nK = p->K[0] * p->K[1] * p->K[2];
  p->Nlr = 1LL * p->lr[0] * p->lr[1] * p->lr[2];
  p->Nout = 1LL * p->out[0] * p->out[1] * p->out[2];
  return PISCO_OK;
}

size_t layout_gram(const Plan& p, void* ws, GramWs* o) {
  Carver c(ws);
  GramWs w{};
  if (p.rows == PISCO_ROWS_VALID) {
    // the explicit rows of C_valid
    w.C = c.take<float2>(size_t(p.Pvalid) * p.n);
    if (o) *o = w;
    return c.used + 256;
  }
  // Forward spectra need two buffers (pass ping-pong); the pair passes need
  // T1 = [P][B0][F1][F2] and T2 = [P][B0][B1][F2].
  const size_t s1 = size_t(p.Q) * p.F[0] * p.F[1] * p.F[2];
  w.S = c.take<float2>(2 * s1);
  w.T1 = c.take<float2>(size_t(p.P) * p.B[0] * p.F[1] * p.F[2]);
  w.T2 = c.take<float2>(size_t(p.P) * p.B[0] * p.B[1] * p.F[2]);
  w.R = c.take<float2>(size_t(p.P) * p.nlag);
  if (o) *o = w;
  return c.used + 256;
}

size_t layout_null(const Plan& p, int b, void* ws, NullWs* o, bool structured) {
  Carver c(ws);
  NullWs w{};
  const size_t nb = size_t(p.n) * b, bb = size_t(b) * b;
  w.X = c.take<double2>(nb);
  w.Z = c.take<double2>(nb);
  w.H = c.take<double2>(bb);
  w.S = c.take<double2>(bb);
  w.U = c.take<double2>(bb);
  w.M = c.take<double2>(bb);
  w.R = c.take<double2>(bb);
  w.dsc = c.take<double>(b);
  w.theta = c.take<double>(b);
  w.filt = c.take<double>(12);
  w.resid = c.take<double>(b);
  // row-chunk partials of the b x b products and residual partials share
  // one buffer (the split-K partials of A X stay in LDS)
  const size_t chunks = (size_t(p.n) + kTnRows - 1) / kTnRows;
  size_t part = chunks * bb;
  const size_t rpart = ((size_t(p.n) + 1023) / 1024) * b;  // doubles
  if (rpart > 2 * part) part = (rpart + 1) / 2;
  w.part = c.take<double2>(part);
  // control words [16], then the device-resident schedule (slot roles and
  // chain skips, 1 + 2 * 60 words)
  w.ctl = c.take<int>(16 + 128);
  w.jac = c.take<double>((size_t(b) + 1) * b * 2);
  w.heev = c.take<double>(heev_workspace_doubles(b));
  if (structured) {
    w.rhat = c.take<double2>(toeplitz_rhat_elems(p));
    w.sp0 = c.take<double2>(toeplitz_spectrum_elems(p, b));
    w.sp1 = c.take<double2>(toeplitz_spectrum_elems(p, b));
  }
  if (o) *o = w;
  return c.used + 256;
}

size_t layout_gx(const Plan& p, int b, void* ws, GxWs* o) {
  Carver c(ws);
  GxWs w{};
  w.Fh = c.take<float2>(size_t(b) * p.Q * p.nK);
  // scratch for the separable passes: filter spectra (b Q planes on the K
  // grid), lag planes (P on the K grid) and the lag -> low-res passes
  size_t half = size_t(b) * p.Q * p.nK;
  const size_t cand[3] = {size_t(p.P) * p.nK, size_t(p.P) * p.B[0] * p.B[1] * p.lr[2],
                          size_t(p.P) * p.B[0] * p.lr[1] * p.lr[2]};
  for (size_t v : cand) half = v > half ? v : half;
  w.tmp_half = half;
  w.Tmp = c.take<float2>(2 * half);
  w.Kh = c.take<float2>(size_t(p.P) * p.nK);
  if (o) *o = w;
  return c.used + 256;
}

int interp_order(const Plan& p, int ord[3]) {
  // the passes of a separable interpolation commute.  x comes last (that pass
  // carries the coil normalisation); of z and y the axis that grows less goes
  // first, which keeps the intermediates small (ties: z first).
  int n = 0;
  if (p.D == 3) {
    const bool zfirst = 1LL * p.out[0] * p.lr[1] <= 1LL * p.out[1] * p.lr[0];
    ord[n++] = zfirst ? 0 : 1;
    ord[n++] = zfirst ? 1 : 0;
  } else {
    ord[n++] = 1;
  }
  ord[n++] = 2;
  return n;
}

size_t layout_maps(const Plan& p, void* ws, MapsWs* o) {
  Carver c(ws);
  MapsWs w{};
  w.rho = c.take<double2>(size_t(p.Q) * p.Nlr);
  const size_t r1 = size_t(p.Q) * p.acs[0] * p.acs[1] * p.lr[2];
  const size_t r2 = size_t(p.Q) * p.acs[0] * p.lr[1] * p.lr[2];
  w.rtA = c.take<double2>(r1 > r2 ? r1 : r2);
  w.rtB = c.take<double2>(r1 > r2 ? r1 : r2);
  w.m = c.take<double2>(p.Nlr);
  w.pmax = c.take<double>((p.Nlr + 255) / 256 + 1);
  // intermediates of the interpolation passes, in the order interp_order gives
  int ord[3];
  const int n = interp_order(p, ord);
  size_t ext[3] = {size_t(p.lr[0]), size_t(p.lr[1]), size_t(p.lr[2])};
  size_t inter[2] = {0, 0};
  for (int i = 0; i + 1 < n; ++i) {
    ext[ord[i]] = size_t(p.out[ord[i]]);
    inter[i] = size_t(p.Q) * ext[0] * ext[1] * ext[2];
  }
  w.tmpA = c.take<float2>(inter[0]);
  w.tmpB = c.take<float2>(inter[1]);
  w.cref = c.take<float2>(size_t(p.Q) * p.Nlr);
  if (o) *o = w;
  return c.used + 256;
}

}  // namespace pisco
