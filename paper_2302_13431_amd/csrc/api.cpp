// extern "C" entry points of libpisco: argument validation, workspace sizing
// and stage chaining.  Kernels live in the .hip translation units.
#include <cstring>
#include <new>

#include "common.hpp"

using namespace pisco;

namespace {

pisco_opts_t default_opts() {
  pisco_opts_t o;
  o.power_iters = 10;  // Sec. IV-E: 10 iterations in the paper's experiments
  o.tol = 0.f;
  o.phase_rule = 0;
  o.block = 0;
  o.max_subspace_iters = 60;
  o.precision = PISCO_PREC_FP32;
  return o;
}

pisco_opts_t resolve(const pisco_opts_t* o) {
  pisco_opts_t r = o ? *o : default_opts();
  if (r.max_subspace_iters <= 0) r.max_subspace_iters = 60;
  return r;
}

int auto_block(const Plan& p) {
  int b = 96;
  const int nr = p.n / 32 * 32;
  if (b > nr) b = nr;
  return b;
}

pisco_status_t fail(Handle* h, pisco_status_t st, const char* msg) {
  if (h) h->last_error = msg;
  return st;
}

bool aligned(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 255u) == 0; }

pisco_status_t check_common(Handle* h, const pisco_problem_t* prob, Plan* plan) {
  if (!h) return PISCO_ERR_ARG;
  std::string err;
  pisco_status_t st = make_plan(prob, plan, &err);
  if (st) {
    h->last_error = err;
    return st;
  }
  return PISCO_OK;
}

pisco_status_t block_of(const Plan& p, const pisco_opts_t& o, int* b, std::string* err) {
  int v = o.block > 0 ? o.block : auto_block(p);
  if (v < 32 || v % 32 != 0) {
    *err = "nullspace block must be a positive multiple of 32 (problem too small?)";
    return PISCO_ERR_UNSUPPORTED;
  }
  if (v > p.n) {
    *err = "nullspace block exceeds the Gram dimension";
    return PISCO_ERR_ARG;
  }
  if (v > 1024) {
    *err = "nullspace block above 1024 is not supported";
    return PISCO_ERR_UNSUPPORTED;
  }
  *b = v;
  return PISCO_OK;
}

size_t ws_stage(const Plan& p, int b, int stage) {
  switch (stage) {
    case PISCO_STAGE_GRAM: return layout_gram(p, nullptr, nullptr);
    case PISCO_STAGE_NULLSPACE: return layout_null(p, b, nullptr, nullptr);
    case PISCO_STAGE_GX: return layout_gx(p, b, nullptr, nullptr);
    case PISCO_STAGE_EIG: return 256;
    case PISCO_STAGE_MAPS: return layout_maps(p, nullptr, nullptr);
    default: return 0;
  }
}

// Intermediates of pisco_estimate followed by the largest stage workspace.
struct EstLayout {
  float2* gram;
  double* eigvals;
  double2* basis;
  int32_t* counts;
  float2* G;
  float2* maps_lr;
  float* lam;
  void* stage_ws;
  size_t total;
};

EstLayout est_layout(const Plan& p, int b, void* ws) {
  Carver c(ws);
  EstLayout e{};
  e.gram = c.take<float2>(size_t(p.n) * p.n);
  e.eigvals = c.take<double>(b);
  e.basis = c.take<double2>(size_t(b) * p.n);
  e.counts = c.take<int32_t>(4);
  e.G = c.take<float2>(size_t(p.P) * p.Nlr);
  e.maps_lr = c.take<float2>(size_t(p.Q) * p.Nlr);
  e.lam = c.take<float>(p.Nlr);
  size_t m = 0;
  for (int st = 1; st <= 5; ++st) {
    const size_t v = ws_stage(p, b, st);
    m = v > m ? v : m;
  }
  e.stage_ws = c.take<char>(m);
  e.total = c.used + 256;
  return e;
}

}  // namespace

extern "C" {

pisco_status_t pisco_create(pisco_handle_t* handle, void* stream) {
  if (!handle) return PISCO_ERR_ARG;
  *handle = nullptr;
  Handle* h = new (std::nothrow) Handle();
  if (!h) return PISCO_ERR_ARG;
  h->stream = static_cast<hipStream_t>(stream);
  hipError_t e = hipMalloc(reinterpret_cast<void**>(&h->status_dev), 64);
  if (e != hipSuccess) {
    delete h;
    return PISCO_ERR_HIP;
  }
  e = hipHostMalloc(reinterpret_cast<void**>(&h->host_pinned), 256, hipHostMallocDefault);
  if (e != hipSuccess) {
    (void)hipFree(h->status_dev);
    delete h;
    return PISCO_ERR_HIP;
  }
  std::memset(h->host_pinned, 0, 256);
  e = hipMemcpy(h->status_dev, h->host_pinned, 64, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipHostFree(h->host_pinned);
    (void)hipFree(h->status_dev);
    delete h;
    return PISCO_ERR_HIP;
  }
  *handle = reinterpret_cast<pisco_handle_t>(h);
  return PISCO_OK;
}

pisco_status_t pisco_destroy(pisco_handle_t handle) {
  Handle* h = reinterpret_cast<Handle*>(handle);
  if (!h) return PISCO_ERR_ARG;
  (void)hipStreamSynchronize(h->stream);
  (void)hipHostFree(h->host_pinned);
  (void)hipFree(h->status_dev);
  delete h;
  return PISCO_OK;
}

pisco_status_t pisco_set_stream(pisco_handle_t handle, void* stream) {
  Handle* h = reinterpret_cast<Handle*>(handle);
  if (!h) return PISCO_ERR_ARG;
  h->stream = static_cast<hipStream_t>(stream);
  return PISCO_OK;
}

const char* pisco_status_string(pisco_status_t st) {
  switch (st) {
    case PISCO_OK: return "ok";
    case PISCO_ERR_ARG: return "invalid argument";
    case PISCO_ERR_WORKSPACE: return "workspace too small";
    case PISCO_ERR_HIP: return "HIP runtime error";
    case PISCO_ERR_UNSUPPORTED: return "unsupported size";
    case PISCO_ERR_NUMERIC: return "numeric failure";
  }
  return "unknown status";
}

const char* pisco_last_error(pisco_handle_t handle) {
  Handle* h = reinterpret_cast<Handle*>(handle);
  return h ? h->last_error.c_str() : "null handle";
}

pisco_status_t pisco_get_status(pisco_handle_t handle, uint32_t* flags) {
  Handle* h = reinterpret_cast<Handle*>(handle);
  if (!h || !flags) return PISCO_ERR_ARG;
  hipError_t e = hipMemcpyAsync(h->host_pinned, h->status_dev, sizeof(uint32_t),
                                hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_check(h, e, "pisco_get_status");
  *flags = h->host_pinned[0];
  h->host_pinned[1] = 0;
  e = hipMemcpyAsync(h->status_dev, h->host_pinned + 1, sizeof(uint32_t),
                     hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_check(h, e, "pisco_get_status");
  return PISCO_OK;
}

pisco_status_t pisco_support(int32_t D, float radius, int32_t* count, int32_t* offsets) {
  if (!count || (D != 2 && D != 3) || !(radius >= 1.0f) || radius > 12.0f)
    return PISCO_ERR_ARG;
  const int n = enumerate_support(D, radius, nullptr, 0);
  *count = n;
  if (offsets) enumerate_support(D, radius, offsets, n);
  return PISCO_OK;
}

pisco_status_t pisco_workspace_size(const pisco_problem_t* prob, const pisco_opts_t* opts,
                                    int32_t stage, size_t* bytes) {
  if (!bytes) return PISCO_ERR_ARG;
  Plan p;
  std::string err;
  pisco_status_t st = make_plan(prob, &p, &err);
  if (st) return st;
  const pisco_opts_t o = resolve(opts);
  int b = 32;
  if (stage == PISCO_STAGE_NULLSPACE || stage == PISCO_STAGE_GX || stage == PISCO_STAGE_ALL) {
    st = block_of(p, o, &b, &err);
    if (st) return st;
  }
  if (stage == PISCO_STAGE_ALL) {
    *bytes = est_layout(p, b, nullptr).total;
    return PISCO_OK;
  }
  if (stage < 1 || stage > 5) return PISCO_ERR_ARG;
  *bytes = ws_stage(p, b, stage);
  return PISCO_OK;
}

pisco_status_t pisco_nullspace_block(const pisco_problem_t* prob, const pisco_opts_t* opts,
                                     int32_t* block) {
  if (!block) return PISCO_ERR_ARG;
  Plan p;
  std::string err;
  pisco_status_t st = make_plan(prob, &p, &err);
  if (st) return st;
  int b = 0;
  st = block_of(p, resolve(opts), &b, &err);
  if (st) return st;
  *block = b;
  return PISCO_OK;
}

pisco_status_t pisco_gram(pisco_handle_t handle, const pisco_problem_t* prob, const void* acs,
                          void* gram, void* ws, size_t ws_bytes) {
  Handle* h = reinterpret_cast<Handle*>(handle);
  Plan p;
  pisco_status_t st = check_common(h, prob, &p);
  if (st) return st;
  if (!acs || !gram || !ws || !aligned(ws)) return fail(h, PISCO_ERR_ARG, "null or unaligned pointer");
  if (ws_bytes < layout_gram(p, nullptr, nullptr))
    return fail(h, PISCO_ERR_WORKSPACE, "workspace too small for pisco_gram");
  return run_gram(h, p, static_cast<const float2*>(acs), static_cast<float2*>(gram), ws);
}

pisco_status_t pisco_nullspace(pisco_handle_t handle, const pisco_problem_t* prob,
                               const pisco_opts_t* opts, const void* gram, double* eigvals,
                               void* basis, int32_t* counts, void* ws, size_t ws_bytes) {
  Handle* h = reinterpret_cast<Handle*>(handle);
  Plan p;
  pisco_status_t st = check_common(h, prob, &p);
  if (st) return st;
  const pisco_opts_t o = resolve(opts);
  int b = 0;
  std::string err;
  if ((st = block_of(p, o, &b, &err))) return fail(h, st, err.c_str());
  if (!gram || !eigvals || !basis || !counts || !ws || !aligned(ws))
    return fail(h, PISCO_ERR_ARG, "null or unaligned pointer");
  if (ws_bytes < layout_null(p, b, nullptr, nullptr))
    return fail(h, PISCO_ERR_WORKSPACE, "workspace too small for pisco_nullspace");
  return run_nullspace(h, p, b, o.max_subspace_iters, static_cast<const float2*>(gram), eigvals,
                       static_cast<double2*>(basis), counts, ws);
}

pisco_status_t pisco_gx(pisco_handle_t handle, const pisco_problem_t* prob,
                        const pisco_opts_t* opts, const void* basis, const int32_t* counts,
                        void* G, void* ws, size_t ws_bytes) {
  Handle* h = reinterpret_cast<Handle*>(handle);
  Plan p;
  pisco_status_t st = check_common(h, prob, &p);
  if (st) return st;
  const pisco_opts_t o = resolve(opts);
  int b = 0;
  std::string err;
  if ((st = block_of(p, o, &b, &err))) return fail(h, st, err.c_str());
  if (!basis || !counts || !G || !ws || !aligned(ws))
    return fail(h, PISCO_ERR_ARG, "null or unaligned pointer");
  if (ws_bytes < layout_gx(p, b, nullptr, nullptr))
    return fail(h, PISCO_ERR_WORKSPACE, "workspace too small for pisco_gx");
  if (o.precision < PISCO_PREC_FP32 || o.precision > PISCO_PREC_SPLIT_BF16)
    return fail(h, PISCO_ERR_ARG, "unknown precision");
  return run_gx(h, p, b, o.precision, static_cast<const double2*>(basis), counts,
                static_cast<float2*>(G), ws);
}

pisco_status_t pisco_eig(pisco_handle_t handle, int32_t Q, int64_t N, float bound,
                         const pisco_opts_t* opts, const void* G, void* maps, float* lam_min,
                         int32_t* iters, void* ws, size_t ws_bytes) {
  return pisco_eig_from(handle, Q, N, bound, opts, G, nullptr, maps, lam_min, iters, ws,
                        ws_bytes);
}

pisco_status_t pisco_eig_from(pisco_handle_t handle, int32_t Q, int64_t N, float bound,
                              const pisco_opts_t* opts, const void* G, const void* init,
                              void* maps, float* lam_min, int32_t* iters, void* ws,
                              size_t ws_bytes) {
  Handle* h = reinterpret_cast<Handle*>(handle);
  (void)ws;
  (void)ws_bytes;
  if (!h) return PISCO_ERR_ARG;
  if (Q < 2 || Q > kMaxQ) return fail(h, PISCO_ERR_ARG, "Q must be in [2, 32]");
  if (N < 0) return fail(h, PISCO_ERR_ARG, "N must be >= 0");
  if (!(bound > 0.f)) return fail(h, PISCO_ERR_ARG, "bound must be positive");
  if (N > 0 && (!G || !maps)) return fail(h, PISCO_ERR_ARG, "null pointer");
  const pisco_opts_t o = resolve(opts);
  if (o.power_iters < 0 || o.power_iters > 100000 || o.tol < 0.f)
    return fail(h, PISCO_ERR_ARG, "bad power-iteration options");
  return run_eig(h, Q, N, bound, o.power_iters, o.tol, static_cast<const float2*>(G),
                 static_cast<const float2*>(init), static_cast<float2*>(maps), lam_min, iters);
}

pisco_status_t pisco_maps(pisco_handle_t handle, const pisco_problem_t* prob,
                          const pisco_opts_t* opts, const void* acs, const void* maps_lr,
                          void* maps_out, void* ws, size_t ws_bytes) {
  Handle* h = reinterpret_cast<Handle*>(handle);
  Plan p;
  pisco_status_t st = check_common(h, prob, &p);
  if (st) return st;
  const pisco_opts_t o = resolve(opts);
  if (o.phase_rule != 0 && o.phase_rule != 1) return fail(h, PISCO_ERR_ARG, "bad phase rule");
  if (!acs || !maps_lr || !maps_out || !ws || !aligned(ws))
    return fail(h, PISCO_ERR_ARG, "null or unaligned pointer");
  if (ws_bytes < layout_maps(p, nullptr, nullptr))
    return fail(h, PISCO_ERR_WORKSPACE, "workspace too small for pisco_maps");
  return run_maps(h, p, o.phase_rule, static_cast<const float2*>(acs),
                  static_cast<const float2*>(maps_lr), static_cast<float2*>(maps_out), ws);
}

pisco_status_t pisco_estimate(pisco_handle_t handle, const pisco_problem_t* prob,
                              const pisco_opts_t* opts, const void* acs, void* maps_out,
                              float* lam_min, void* ws, size_t ws_bytes) {
  Handle* h = reinterpret_cast<Handle*>(handle);
  Plan p;
  pisco_status_t st = check_common(h, prob, &p);
  if (st) return st;
  const pisco_opts_t o = resolve(opts);
  int b = 0;
  std::string err;
  if ((st = block_of(p, o, &b, &err))) return fail(h, st, err.c_str());
  if (!acs || !maps_out || !ws || !aligned(ws))
    return fail(h, PISCO_ERR_ARG, "null or unaligned pointer");
  if (o.precision < PISCO_PREC_FP32 || o.precision > PISCO_PREC_SPLIT_BF16)
    return fail(h, PISCO_ERR_ARG, "unknown precision");
  EstLayout e = est_layout(p, b, ws);
  if (ws_bytes < e.total) return fail(h, PISCO_ERR_WORKSPACE, "workspace too small for pisco_estimate");
  const float2* a = static_cast<const float2*>(acs);
  if ((st = run_gram(h, p, a, e.gram, e.stage_ws))) return st;
  if ((st = run_nullspace(h, p, b, o.max_subspace_iters, e.gram, e.eigvals, e.basis, e.counts,
                          e.stage_ws)))
    return st;
  if ((st = run_gx(h, p, b, o.precision, e.basis, e.counts, e.G, e.stage_ws))) return st;
  float* lam = lam_min ? lam_min : e.lam;
  if ((st = run_eig(h, p.Q, p.Nlr, float(p.L), o.power_iters, o.tol, e.G, nullptr, e.maps_lr, lam,
                    nullptr)))
    return st;
  return run_maps(h, p, o.phase_rule, a, e.maps_lr, static_cast<float2*>(maps_out),
                  e.stage_ws);
}

}  // extern "C"
