// extern "C" entry points of libpisco: argument validation, workspace sizing
// and stage chaining.  Kernels live in the .hip translation units.
#include <cstdio>
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
  o.schedule = PISCO_SCHED_AUTO;
  o.product = PISCO_PRODUCT_AUTO;
  return o;
}

pisco_opts_t resolve(const pisco_opts_t* o) {
  pisco_opts_t r = o ? *o : default_opts();
  if (r.max_subspace_iters <= 0) r.max_subspace_iters = 60;
  return r;
}

// Automatic nullspace block: the signal rank of calibration Grams measured
// here is 0.5 to 0.9 |Lambda| (21 of 29, 71 of 81, 157 of 257, 263 of 515
// support points), so the block is 0.6 |Lambda| + 32 rounded up to a
// multiple of 32 (64 at least), within the Gram dimension and 1024.
int auto_block(const Plan& p) {
  int b = (int(0.6 * p.L) + 32 + 31) / 32 * 32;
  b = b < 64 ? 64 : (b > 1024 ? 1024 : b);
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

// Stage scratch without tables (pisco_estimate's shared stage region).
size_t ws_stage_scratch(const Plan& p, int b, int stage) {
  switch (stage) {
    case PISCO_STAGE_GRAM: return layout_gram(p, nullptr, nullptr);
    case PISCO_STAGE_NULLSPACE: return layout_null(p, b, nullptr, nullptr);
    case PISCO_STAGE_GX: return layout_gx(p, b, nullptr, nullptr);
    case PISCO_STAGE_EIG: return 256;
    case PISCO_STAGE_MAPS: return layout_maps(p, nullptr, nullptr);
    case PISCO_STAGE_MASK: return layout_mask(p, nullptr, nullptr, nullptr, nullptr);
    default: return 0;
  }
}

unsigned stage_tables(int stage) {
  switch (stage) {
    case PISCO_STAGE_GRAM: return kTabSupport;
    case PISCO_STAGE_GX: return kTabGx;
    case PISCO_STAGE_MAPS: return kTabMaps;
    case PISCO_STAGE_MASK: return kTabMask;
    default: return 0;
  }
}

// A stage call's workspace: its tables, then its scratch.
size_t ws_stage(const Plan& p, int b, int stage) {
  const unsigned tb = stage_tables(stage);
  const size_t tabs = tb ? (layout_tables(p, tb, nullptr, nullptr) + 255) & ~size_t(255) : 0;
  return tabs + ws_stage_scratch(p, b, stage);
}

// Carves a stage call's tables from the front of ws, builds them and returns
// the scratch that follows.
pisco_status_t stage_prologue(Handle* h, const Plan& p, int stage, void* ws, Tables* t,
                              void** scratch) {
  const unsigned tb = stage_tables(stage);
  const size_t tabs = (layout_tables(p, tb, ws, t) + 255) & ~size_t(255);
  *scratch = static_cast<char*>(ws) + tabs;
  return build_tables(h, p, tb, *t);
}

// Intermediates of pisco_estimate followed by the largest stage workspace.
struct EstLayout {
  Tables tabs;
  float2* gram;
  double* eigvals;
  double2* basis;
  int32_t* counts;
  float2* G;
  float2* maps_lr;
  float* lam;
  void* null_ws;
  void* stage_ws;
  size_t total;
};

EstLayout est_layout(const Plan& p, int b, void* ws, bool structured) {
  Carver c(ws);
  EstLayout e{};
  // tables first: their offsets do not depend on the block size
  char* tb = c.take<char>(layout_tables(p, kTabAll, nullptr, nullptr));
  layout_tables(p, kTabAll, tb, &e.tabs);
  // the explicit Gram, or (structured products) only its lags
  e.gram = c.take<float2>(structured ? size_t(p.P) * p.nlag : size_t(p.n) * p.n);
  e.eigvals = c.take<double>(b);
  e.basis = c.take<double2>(size_t(b) * p.n);
  e.counts = c.take<int32_t>(4);
  e.G = c.take<float2>(size_t(p.P) * p.Nlr);
  e.maps_lr = c.take<float2>(size_t(p.Q) * p.Nlr);
  e.lam = c.take<float>(p.Nlr);
  // the nullspace stage has a region of its own: the later stages may be
  // enqueued while its iteration can still go on
  e.null_ws = c.take<char>(layout_null(p, b, nullptr, nullptr, structured));
  size_t m = 0;
  for (int st = 1; st <= 5; ++st) {
    const size_t v = st == 2 ? 0 : ws_stage_scratch(p, b, st);
    m = v > m ? v : m;
  }
  e.stage_ws = c.take<char>(m);
  e.total = c.used + 256;
  return e;
}

}  // namespace

namespace pisco {

bool structured_product(const Plan& p, const pisco_opts_t& o) {
  if (p.rows != PISCO_ROWS_ALL) return false;  // the masked Gram has no lag structure
  if (o.product == PISCO_PRODUCT_STRUCTURED) return true;
  if (o.product == PISCO_PRODUCT_DENSE) return false;
  return p.D == 3 && p.n >= 4096;
}


size_t estimate_ws_size(const Plan& p, int b, bool structured) {
  return est_layout(p, b, nullptr, structured).total;
}

pisco_status_t choose_schedule(Handle* h, const pisco_opts_t& o, int* device_products) {
  *device_products = 0;
  if (o.schedule != PISCO_SCHED_AUTO && o.schedule != PISCO_SCHED_DEVICE) {
    h->last_error = "unknown nullspace schedule";
    return PISCO_ERR_ARG;
  }
  bool device = o.schedule == PISCO_SCHED_DEVICE;
  if (!device) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    const hipError_t e = hipStreamIsCapturing(h->stream, &cs);
    if (e != hipSuccess) return hip_check(h, e, "schedule: capture query");
    device = cs != hipStreamCaptureStatusNone;
  }
  if (device) {
    const int cap = o.max_subspace_iters < kDeviceProducts ? o.max_subspace_iters : kDeviceProducts;
    *device_products = cap < 4 ? 4 : cap;
  }
  return PISCO_OK;
}

pisco_status_t estimate_core(Handle* h, const Plan& p, const pisco_opts_t& o, int b,
                             const float2* acs, float2* maps_out, float* lam_min, void* ws,
                             int fixed_products, int ax_waves, int32_t** counts_out,
                             bool tables_ready) {
  const bool structured = structured_product(p, o);
  EstLayout e = est_layout(p, b, ws, structured);
  if (counts_out) *counts_out = e.counts;
  pisco_status_t st;
  int device_products = 0;
  if (fixed_products <= 0 && (st = choose_schedule(h, o, &device_products))) return st;
  if (!tables_ready && (st = build_tables(h, p, kTabAll, e.tabs))) return st;
  if ((st = run_gram(h, p, e.tabs, acs, e.gram, e.stage_ws, structured ? e.gram : nullptr)))
    return st;
  ToeplitzOp tp{};
  if (structured) {
    NullWs nw;
    layout_null(p, b, e.null_ws, &nw, true);
    tp.lags = e.gram;
    tp.boxmap = e.tabs.boxmap;
    tp.sup = e.tabs.sup;
    tp.Tf = e.tabs.Tf;
    tp.Ti = e.tabs.Ti;
    tp.Tr = e.tabs.Tr;
    tp.rhat = nw.rhat;
    tp.buf0 = nw.sp0;
    tp.buf1 = nw.sp1;
    tp.D = p.D;
    tp.W = 2 * p.tau + 1;
    tp.Wz = p.D == 3 ? tp.W : 1;
    tp.F = p.K[2];
    tp.Fz = p.K[0];
    tp.Q = p.Q;
    tp.L = p.L;
    tp.P = p.P;
  }
  float* lam = lam_min ? lam_min : e.lam;
  const std::function<pisco_status_t()> later = [&]() -> pisco_status_t {
    pisco_status_t s2;
    if ((s2 = run_gx(h, p, e.tabs, b, o.precision, e.basis, e.counts, e.G, e.stage_ws)))
      return s2;
    if ((s2 = run_eig(h, p.Q, p.Nlr, float(p.L), o.power_iters, o.tol, e.G, nullptr,
                      e.maps_lr, lam, nullptr)))
      return s2;
    return run_maps(h, p, e.tabs, o.phase_rule, acs, e.maps_lr, maps_out, e.stage_ws);
  };
  bool queued = false;
  if ((st = run_nullspace(h, p, b, o.max_subspace_iters, e.gram, e.eigvals, e.basis, e.counts,
                          e.null_ws, fixed_products, ax_waves, &later, &queued,
                          device_products, structured ? &tp : nullptr)))
    return st;
  return queued ? PISCO_OK : later();
}

}  // namespace pisco

extern "C" {

pisco_status_t pisco_create(pisco_handle_t* handle, void* stream) {
  if (!handle) return PISCO_ERR_ARG;
  *handle = nullptr;
  Handle* h = new (std::nothrow) Handle();
  if (!h) return PISCO_ERR_ARG;
  h->stream = static_cast<hipStream_t>(stream);
  {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        cus > 0)
      h->num_cu = cus;
  }
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
  if (e == hipSuccess)
    e = hipHostMalloc(reinterpret_cast<void**>(&h->host_ctl), 64, hipHostMallocCoherent);
  if (e == hipSuccess) {
    std::memset(h->host_ctl, 0, 64);
    e = hipHostGetDevicePointer(reinterpret_cast<void**>(&h->host_ctl_dev), h->host_ctl, 0);
  }
  if (e != hipSuccess) {
    if (h->host_ctl) (void)hipHostFree(h->host_ctl);
    (void)hipHostFree(h->host_pinned);
    (void)hipFree(h->status_dev);
    delete h;
    return PISCO_ERR_HIP;
  }
  // resolve the static scratch of pisco_gram_static on the current device
  void* scratch_ptr = nullptr;
  if (gram_scratch_address(h, &scratch_ptr) != PISCO_OK) {
    (void)hipHostFree(h->host_ctl);
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
  if (h->sched_ev) (void)hipEventDestroy(h->sched_ev);
  (void)hipHostFree(h->host_ctl);
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

pisco_status_t pisco_support(int32_t D, float radius, int32_t shape, int32_t* count,
                             int32_t* offsets) {
  if (!count || (D != 2 && D != 3) || !(radius >= 1.0f) || radius > 12.0f)
    return PISCO_ERR_ARG;
  if (shape != PISCO_SHAPE_ELLIPSOID && shape != PISCO_SHAPE_RECTANGLE) return PISCO_ERR_ARG;
  const int n = enumerate_support(D, radius, shape, nullptr, 0);
  *count = n;
  if (offsets) enumerate_support(D, radius, shape, offsets, n);
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
    *bytes = est_layout(p, b, nullptr, structured_product(p, o)).total;
    return PISCO_OK;
  }
  if (stage < 1 || stage > 6) return PISCO_ERR_ARG;
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
  if (ws_bytes < ws_stage(p, 0, PISCO_STAGE_GRAM))
    return fail(h, PISCO_ERR_WORKSPACE, "workspace too small for pisco_gram");
  Tables t;
  void* scratch = nullptr;
  if ((st = stage_prologue(h, p, PISCO_STAGE_GRAM, ws, &t, &scratch))) return st;
  return run_gram(h, p, t, static_cast<const float2*>(acs), static_cast<float2*>(gram), scratch);
}

pisco_status_t pisco_gram_static(pisco_handle_t handle, const pisco_problem_t* prob,
                                 const void* acs, void* gram) {
  Handle* h = reinterpret_cast<Handle*>(handle);
  Plan p;
  pisco_status_t st = check_common(h, prob, &p);
  if (st) return st;
  if (!acs || !gram) return fail(h, PISCO_ERR_ARG, "null pointer");
  return run_gram_static(h, p, static_cast<const float2*>(acs), static_cast<float2*>(gram));
}

pisco_status_t pisco_gram_static_bytes(const pisco_problem_t* prob, size_t* bytes,
                                       size_t* limit) {
  if (!bytes && !limit) return PISCO_ERR_ARG;
  Plan p;
  std::string err;
  pisco_status_t st = make_plan(prob, &p, &err);
  if (st) return st;
  if (bytes) *bytes = gram_static_bytes(p);
  if (limit) *limit = kGramScratchBytes;
  return PISCO_OK;
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
  int device_products = 0;
  if ((st = choose_schedule(h, o, &device_products))) return st;
  return run_nullspace(h, p, b, o.max_subspace_iters, static_cast<const float2*>(gram), eigvals,
                       static_cast<double2*>(basis), counts, ws, 0, 0, nullptr, nullptr, device_products);
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
  if (ws_bytes < ws_stage(p, b, PISCO_STAGE_GX))
    return fail(h, PISCO_ERR_WORKSPACE, "workspace too small for pisco_gx");
  if (o.precision < PISCO_PREC_FP32 || o.precision > PISCO_PREC_SPLIT_BF16)
    return fail(h, PISCO_ERR_ARG, "unknown precision");
  Tables t;
  void* scratch = nullptr;
  if ((st = stage_prologue(h, p, PISCO_STAGE_GX, ws, &t, &scratch))) return st;
  return run_gx(h, p, t, b, o.precision, static_cast<const double2*>(basis), counts,
                static_cast<float2*>(G), scratch);
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
  return pisco_eig_checked(handle, Q, N, bound, opts, G, init, maps, lam_min, iters, nullptr,
                           nullptr, ws, ws_bytes);
}

pisco_status_t pisco_eig_checked(pisco_handle_t handle, int32_t Q, int64_t N, float bound,
                                 const pisco_opts_t* opts, const void* G, const void* init,
                                 void* maps, float* lam_min, int32_t* iters, double* lam64,
                                 double* resid64, void* ws, size_t ws_bytes) {
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
                 static_cast<const float2*>(init), static_cast<float2*>(maps), lam_min, iters,
                 lam64, resid64);
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
  if (ws_bytes < ws_stage(p, 0, PISCO_STAGE_MAPS))
    return fail(h, PISCO_ERR_WORKSPACE, "workspace too small for pisco_maps");
  Tables t;
  void* scratch = nullptr;
  if ((st = stage_prologue(h, p, PISCO_STAGE_MAPS, ws, &t, &scratch))) return st;
  return run_maps(h, p, t, o.phase_rule, static_cast<const float2*>(acs),
                  static_cast<const float2*>(maps_lr), static_cast<float2*>(maps_out), scratch);
}

pisco_status_t pisco_eig_sets_workspace_size(int32_t Q, int64_t N, size_t* bytes) {
  if (!bytes || Q < 2 || Q > kMaxQ || N < 0) return PISCO_ERR_ARG;
  *bytes = layout_eig_sets(Q, N);
  return PISCO_OK;
}

pisco_status_t pisco_eig_sets(pisco_handle_t handle, int32_t Q, int64_t N, float bound,
                              int32_t sets, int32_t krylov, const void* G, void* maps,
                              float* lam, float* resid, void* ws, size_t ws_bytes) {
  Handle* h = reinterpret_cast<Handle*>(handle);
  if (!h) return PISCO_ERR_ARG;
  if (Q < 2 || Q > kMaxQ) return fail(h, PISCO_ERR_ARG, "Q must be in [2, 32]");
  if (N < 0) return fail(h, PISCO_ERR_ARG, "N must be >= 0");
  if (!(bound > 0.f) && !(bound <= 0.f)) return fail(h, PISCO_ERR_ARG, "bound must be a number");
  if (krylov < 1 || krylov > Q) return fail(h, PISCO_ERR_ARG, "krylov must be in [1, Q]");
  if (sets < 1 || sets > 8 || sets > krylov)
    return fail(h, PISCO_ERR_ARG, "sets must be in [1, min(8, krylov)]");
  if (N > 0 && (!G || !maps || !lam || !ws || !aligned(ws)))
    return fail(h, PISCO_ERR_ARG, "null or unaligned pointer");
  if (ws_bytes < layout_eig_sets(Q, N))
    return fail(h, PISCO_ERR_WORKSPACE, "workspace too small for pisco_eig_sets");
  return run_eig_sets(h, Q, N, bound, krylov, sets, static_cast<const float2*>(G),
                      static_cast<float2*>(maps), lam, resid, ws);
}

pisco_status_t pisco_llr_workspace_size(int64_t B, int32_t Q, int32_t rank, size_t* bytes) {
  if (!bytes || B < 0 || Q < 2 || Q > kMaxQ || rank < 1 || rank > 8 || rank > Q)
    return PISCO_ERR_ARG;
  *bytes = layout_llr(B, Q, rank, nullptr, nullptr, nullptr, nullptr);
  return PISCO_OK;
}

pisco_status_t pisco_llr_svd(pisco_handle_t handle, int64_t B, int32_t m, int32_t Q,
                             int32_t rank, const void* X, float* sigma, void* V, void* Xr,
                             void* ws, size_t ws_bytes) {
  Handle* h = reinterpret_cast<Handle*>(handle);
  if (!h) return PISCO_ERR_ARG;
  if (B < 0 || m < 1) return fail(h, PISCO_ERR_ARG, "need B >= 0 and m >= 1");
  if (B > 0x7fffffffLL) return fail(h, PISCO_ERR_ARG, "B must be < 2^31 (one workgroup per patch)");
  if (Q < 2 || Q > kMaxQ) return fail(h, PISCO_ERR_ARG, "Q must be in [2, 32]");
  if (rank < 1 || rank > 8 || rank > Q) return fail(h, PISCO_ERR_ARG, "rank must be in [1, min(8, Q)]");
  if (B > 0 && (!X || !sigma || !ws || !aligned(ws)))
    return fail(h, PISCO_ERR_ARG, "null or unaligned pointer");
  if (ws_bytes < layout_llr(B, Q, rank, nullptr, nullptr, nullptr, nullptr))
    return fail(h, PISCO_ERR_WORKSPACE, "workspace too small for pisco_llr_svd");
  return run_llr(h, B, m, Q, rank, static_cast<const float2*>(X), sigma,
                 static_cast<float2*>(V), static_cast<float2*>(Xr), ws);
}

pisco_status_t pisco_support_mask(pisco_handle_t handle, const pisco_problem_t* prob,
                                  const float* lam_min, float thresh, uint8_t* mask, void* ws,
                                  size_t ws_bytes) {
  Handle* h = reinterpret_cast<Handle*>(handle);
  Plan p;
  pisco_status_t st = check_common(h, prob, &p);
  if (st) return st;
  if (!lam_min || !mask || !ws || !aligned(ws))
    return fail(h, PISCO_ERR_ARG, "null or unaligned pointer");
  if (!(thresh > 0.f) || !(thresh < 1.f)) return fail(h, PISCO_ERR_ARG, "thresh must be in (0, 1)");
  if (ws_bytes < ws_stage(p, 0, PISCO_STAGE_MASK))
    return fail(h, PISCO_ERR_WORKSPACE, "workspace too small for pisco_support_mask");
  Tables t;
  void* scratch = nullptr;
  if ((st = stage_prologue(h, p, PISCO_STAGE_MASK, ws, &t, &scratch))) return st;
  return run_support_mask(h, p, t, lam_min, float(p.L), thresh, mask, scratch);
}

pisco_status_t pisco_espirit_operator(pisco_handle_t handle, int32_t Q, int64_t N, float bound,
                                      const void* G, void* B) {
  Handle* h = reinterpret_cast<Handle*>(handle);
  if (!h) return PISCO_ERR_ARG;
  if (Q < 2 || Q > kMaxQ) return fail(h, PISCO_ERR_ARG, "Q must be in [2, 32]");
  if (N < 0) return fail(h, PISCO_ERR_ARG, "N must be >= 0");
  if (!(bound > 0.f)) return fail(h, PISCO_ERR_ARG, "bound must be positive");
  if (N > 0 && (!G || !B)) return fail(h, PISCO_ERR_ARG, "null pointer");
  return run_espirit_operator(h, Q, N, bound, static_cast<const float2*>(G),
                              static_cast<float2*>(B));
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
  if (o.product < PISCO_PRODUCT_AUTO || o.product > PISCO_PRODUCT_STRUCTURED)
    return fail(h, PISCO_ERR_ARG, "unknown product");
  if (ws_bytes < estimate_ws_size(p, b, structured_product(p, o)))
    return fail(h, PISCO_ERR_WORKSPACE, "workspace too small for pisco_estimate");
  return estimate_core(h, p, o, b, static_cast<const float2*>(acs),
                       static_cast<float2*>(maps_out), lam_min, ws, 0, 0);
}

}  // extern "C"

// ---------------------------------------------------------------- batches

struct BatchSlice {
  Plan p;
  pisco_opts_t o;
  int b = 0, products = 0, ax_waves = 0;
  int bmax = 0;        // widest block the slice's workspace region holds
  size_t ws_bytes = 0;  // size of that region
  const float2* acs = nullptr;
  float2* out = nullptr;
  float* lam = nullptr;
  void* ws = nullptr;
};

struct pisco_batch_s {
  Handle* h = nullptr;
  std::vector<hipStream_t> streams;
  std::vector<Handle*> sub;
  std::vector<hipEvent_t> events;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<BatchSlice> slices;
};

namespace {

std::string shape_key(const Plan& p, const pisco_opts_t& o) {
  char buf[256];
  std::snprintf(buf, sizeof(buf), "%d:%d:%d,%d,%d:%.4f:%d,%d,%d:%d,%d,%d:%.5f:%d:%d:%.3g:%d",
                p.D, p.Q, p.acs[0], p.acs[1], p.acs[2], p.radius, p.lr[0], p.lr[1], p.lr[2],
                p.out[0], p.out[1], p.out[2], p.thresh, o.precision, o.power_iters, o.tol,
                o.phase_rule);
  return buf;
}

// Device status flags read back and cleared (synchronises the stream).
pisco_status_t take_flags(Handle* h, uint32_t* flags) {
  return pisco_get_status(reinterpret_cast<pisco_handle_t>(h), flags);
}

// Largest nullspace block the tuner may try (the workspace is sized for it):
// the automatic block plus 96, within the Gram dimension and 1024.
int max_block(const Plan& p, int b0) {
  const int cap = p.n / 32 * 32 < 1024 ? p.n / 32 * 32 : 1024;
  return b0 + 96 <= cap ? b0 + 96 : (cap > b0 ? cap : b0);
}

pisco_status_t batch_prepare(Handle* h, int32_t B, const pisco_problem_t* probs,
                             const pisco_opts_t* opts, std::vector<BatchSlice>* out,
                             size_t* total) {
  if (B < 1 || !probs) return fail(h, PISCO_ERR_ARG, "batch: empty or null problem list");
  size_t sum = 0;
  out->clear();
  for (int i = 0; i < B; ++i) {
    BatchSlice sl;
    pisco_status_t st = check_common(h, &probs[i], &sl.p);
    if (st) return st;
    sl.o = resolve(opts ? &opts[i] : nullptr);
    std::string err;
    if ((st = block_of(sl.p, sl.o, &sl.b, &err))) return fail(h, st, err.c_str());
    if (sl.o.precision < PISCO_PREC_FP32 || sl.o.precision > PISCO_PREC_SPLIT_BF16)
      return fail(h, PISCO_ERR_ARG, "unknown precision");
    sl.bmax = sl.o.block > 0 ? sl.b : max_block(sl.p, sl.b);
    if (sl.o.product < PISCO_PRODUCT_AUTO || sl.o.product > PISCO_PRODUCT_STRUCTURED)
      return fail(h, PISCO_ERR_ARG, "unknown product");
    sl.ws_bytes = (estimate_ws_size(sl.p, sl.bmax, structured_product(sl.p, sl.o)) + 255) &
                  ~size_t(255);
    sum += sl.ws_bytes;
    out->push_back(sl);
  }
  *total = sum;
  return PISCO_OK;
}

void batch_free(pisco_batch_s* bt) {
  if (!bt) return;
  if (bt->exec) (void)hipGraphExecDestroy(bt->exec);
  if (bt->graph) (void)hipGraphDestroy(bt->graph);
  for (hipEvent_t e : bt->events) (void)hipEventDestroy(e);
  for (Handle* s : bt->sub) {  // status word and pinned buffers are borrowed
    if (s->sched_ev) (void)hipEventDestroy(s->sched_ev);
    delete s;
  }
  for (hipStream_t s : bt->streams) (void)hipStreamDestroy(s);
  delete bt;
}

}  // namespace

extern "C" {

pisco_status_t pisco_batch_workspace_size(int32_t B, const pisco_problem_t* probs,
                                          const pisco_opts_t* opts, size_t* bytes) {
  Handle tmp;
  std::vector<BatchSlice> sl;
  if (!bytes) return PISCO_ERR_ARG;
  return batch_prepare(&tmp, B, probs, opts, &sl, bytes);
}

pisco_status_t pisco_batch_create(pisco_handle_t handle, int32_t B, const pisco_problem_t* probs,
                                  const pisco_opts_t* opts, const void* const* acs,
                                  void* const* maps_out, float* const* lam_min, void* ws,
                                  size_t ws_bytes, pisco_batch_t* batch) {
  Handle* h = reinterpret_cast<Handle*>(handle);
  if (!h || !batch) return PISCO_ERR_ARG;
  *batch = nullptr;
  std::vector<BatchSlice> sl;
  size_t need = 0;
  pisco_status_t st = batch_prepare(h, B, probs, opts, &sl, &need);
  if (st) return st;
  if (!acs || !maps_out || !ws || !aligned(ws))
    return fail(h, PISCO_ERR_ARG, "batch: null or unaligned pointer");
  if (ws_bytes < need) return fail(h, PISCO_ERR_WORKSPACE, "batch: workspace too small");
  char* base = static_cast<char*>(ws);
  for (int i = 0; i < B; ++i) {
    if (!acs[i] || !maps_out[i]) return fail(h, PISCO_ERR_ARG, "batch: null slice pointer");
    sl[i].acs = static_cast<const float2*>(acs[i]);
    sl[i].out = static_cast<float2*>(maps_out[i]);
    sl[i].lam = lam_min ? lam_min[i] : nullptr;
    sl[i].ws = base;
    base += sl[i].ws_bytes;
  }
  // every run of a slice checks that its block fits the slice's region
  auto run = [&](const BatchSlice& x, Handle* hh, int bb, int fixed, int waves,
                 int32_t** counts, bool tables_ready = false) -> pisco_status_t {
    if (bb > x.bmax || estimate_ws_size(x.p, bb, structured_product(x.p, x.o)) > x.ws_bytes)
      return fail(h, PISCO_ERR_WORKSPACE, "batch: block exceeds the slice's workspace region");
    return estimate_core(hh, x.p, x.o, bb, x.acs, x.out, x.lam, x.ws, fixed, waves, counts,
                         tables_ready);
  };
  uint32_t saved = 0, flags = 0, tune_flags = 0;
  if ((st = take_flags(h, &saved))) return st;
  hipEvent_t t0 = nullptr, t1 = nullptr;
  hipError_t e = hipEventCreate(&t0);
  if (e == hipSuccess) e = hipEventCreate(&t1);
  if (e != hipSuccess) return hip_check(h, e, "batch: events");
  auto cleanup_events = [&]() {
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
  };
  const uint32_t bad = PISCO_FLAG_NONFINITE | PISCO_FLAG_NOT_CONVERGED | PISCO_FLAG_BLOCK_TOO_SMALL;
  // autotune per shape (timed eager runs), then one eager planning run per
  // slice that fixes its product count
  for (int i = 0; i < B; ++i) {
    BatchSlice& x = sl[i];
    const std::string key = shape_key(x.p, x.o) + (x.o.block > 0 ? ":b" + std::to_string(x.b) : "");
    auto it = h->tuned.find(key);
    if (it == h->tuned.end()) {
      std::vector<int> blocks{x.b};
      const int bcap = x.bmax;
      if (x.b + 32 <= bcap) blocks.push_back(x.b + 32);
      const int waves[3] = {1024, 2048, 4096};
      float best = 3.0e38f;
      std::pair<int, int> choice(x.b, 2048);
      bool found = false;
      for (size_t bi = 0; bi < blocks.size(); ++bi) {
        const int bb = blocks[bi];
        for (int wv : waves) {
          float ms = 0.f;
          for (int rep = 0; rep < 2 && !st; ++rep) {
            if (rep == 1) e = hipEventRecord(t0, h->stream);
            st = run(x, h, bb, 0, wv, nullptr);
            if (rep == 1 && e == hipSuccess) e = hipEventRecord(t1, h->stream);
          }
          if (st) {
            cleanup_events();
            return st;
          }
          if (e == hipSuccess) e = hipEventSynchronize(t1);
          if (e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1);
          if (e != hipSuccess) {
            cleanup_events();
            return hip_check(h, e, "batch: tuning");
          }
          if ((st = take_flags(h, &tune_flags))) {
            cleanup_events();
            return st;
          }
          if (!(tune_flags & bad) && ms < best) {
            best = ms;
            choice = std::make_pair(bb, wv);
            found = true;
          }
        }
        // no candidate converged yet (signal rank at the block size): widen
        if (!found && bi + 1 == blocks.size() && bb + 32 <= bcap) blocks.push_back(bb + 32);
      }
      it = h->tuned.emplace(key, choice).first;
    }
    // a shape's cached choice was tuned within the same bmax (same shape key)
    x.b = it->second.first < x.bmax ? it->second.first : x.bmax;
    x.ax_waves = it->second.second;
    // planning run; the signal rank depends on the data, so a slice whose
    // rank reaches the tuned block gets a wider block of its own, up to the
    // block its workspace region was sized for
    const int bcap = x.bmax;
    uint32_t plan_flags = 0;
    while (true) {
      int32_t* counts = nullptr;
      if ((st = run(x, h, x.b, 0, x.ax_waves, &counts))) {
        cleanup_events();
        return st;
      }
      int32_t hc[4] = {0, 0, 0, 0};
      e = hipMemcpyAsync(hc, counts, sizeof(hc), hipMemcpyDeviceToHost, h->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
      if (e != hipSuccess) {
        cleanup_events();
        return hip_check(h, e, "batch: planning");
      }
      if ((st = take_flags(h, &plan_flags))) {
        cleanup_events();
        return st;
      }
      // one product beyond the eager run's count: the fixed schedule has a
      // single Rayleigh-Ritz step where the eager run may have had two
      x.products = (hc[2] > 3 ? hc[2] : 3) + 1;
      if (!(plan_flags & PISCO_FLAG_BLOCK_TOO_SMALL) || x.b + 32 > bcap) break;
      x.b += 32;
    }
    flags |= plan_flags;
  }
  cleanup_events();
  // restore the flags the caller had not read yet, plus those of the
  // planning runs (the tuning runs' flags only steered the choice)
  h->host_pinned[2] = saved | flags;
  e = hipMemcpyAsync(h->status_dev, h->host_pinned + 2, sizeof(uint32_t), hipMemcpyHostToDevice,
                     h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_check(h, e, "batch: flags");

  // capture: the slices spread over a few streams (default priority) that
  // fork from and join back into the first one
  pisco_batch_s* bt = new (std::nothrow) pisco_batch_s();
  if (!bt) return fail(h, PISCO_ERR_ARG, "batch: out of host memory");
  bt->h = h;
  bt->slices = sl;
  const int S = B < 4 ? B : 4;
  for (int k = 0; k < S && e == hipSuccess; ++k) {
    hipStream_t s = nullptr;
    e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e == hipSuccess) {
      bt->streams.push_back(s);
      Handle* sh = new Handle();
      sh->stream = s;
      sh->status_dev = h->status_dev;
      sh->host_pinned = h->host_pinned;
      sh->host_ctl = h->host_ctl;
      sh->host_ctl_dev = h->host_ctl_dev;
      bt->sub.push_back(sh);
    }
  }
  for (int k = 0; k < S + 1 && e == hipSuccess; ++k) {
    hipEvent_t ev = nullptr;
    e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e == hipSuccess) bt->events.push_back(ev);
  }
  if (e != hipSuccess) {
    batch_free(bt);
    return hip_check(h, e, "batch: streams");
  }
  hipStream_t origin = bt->streams[0];
  e = hipStreamBeginCapture(origin, hipStreamCaptureModeRelaxed);
  if (e == hipSuccess) e = hipEventRecord(bt->events[0], origin);
  for (int k = 1; k < S && e == hipSuccess; ++k) e = hipStreamWaitEvent(bt->streams[k], bt->events[0], 0);
  for (int i = 0; i < B && e == hipSuccess && !st; ++i) {
    const BatchSlice& x = bt->slices[i];
    // the slice's planning run built its tables in its region (at the front
    // of the layout, whatever the block): the graph does not rebuild them
    st = run(x, bt->sub[i % S], x.b, x.products, x.ax_waves, nullptr, true);
  }
  for (int k = 1; k < S && e == hipSuccess; ++k) {
    e = hipEventRecord(bt->events[k], bt->streams[k]);
    if (e == hipSuccess) e = hipStreamWaitEvent(origin, bt->events[k], 0);
  }
  hipGraph_t g = nullptr;
  const hipError_t e_end = hipStreamEndCapture(origin, &g);
  bt->graph = g;
  if (e == hipSuccess) e = e_end;
  if (st || e != hipSuccess) {
    batch_free(bt);
    if (st) return st;
    return hip_check(h, e, "batch: capture");
  }
  e = hipGraphInstantiate(&bt->exec, bt->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    batch_free(bt);
    return hip_check(h, e, "batch: instantiate");
  }
  *batch = bt;
  return PISCO_OK;
}

pisco_status_t pisco_batch_launch(pisco_batch_t batch) {
  if (!batch || !batch->exec) return PISCO_ERR_ARG;
  const hipError_t e = hipGraphLaunch(batch->exec, batch->h->stream);
  return hip_check(batch->h, e, "pisco_batch_launch");
}

pisco_status_t pisco_batch_slice_info(pisco_batch_t batch, int32_t i, int32_t* block,
                                      int32_t* products, int32_t* ax_waves) {
  if (!batch || i < 0 || i >= int32_t(batch->slices.size())) return PISCO_ERR_ARG;
  const BatchSlice& x = batch->slices[i];
  if (block) *block = x.b;
  if (products) *products = x.products;
  if (ax_waves) *ax_waves = x.ax_waves;
  return PISCO_OK;
}

pisco_status_t pisco_batch_destroy(pisco_batch_t batch) {
  if (!batch) return PISCO_ERR_ARG;
  (void)hipStreamSynchronize(batch->h->stream);
  for (hipStream_t s : batch->streams) (void)hipStreamSynchronize(s);
  batch_free(batch);
  return PISCO_OK;
}

}  // extern "C"
