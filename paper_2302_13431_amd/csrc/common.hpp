// Internal definitions shared by the HIP translation units of libpisco.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <functional>
#include <map>
#include <string>
#include <vector>

#include "pisco.h"

namespace pisco {

// ------------------------------------------------------------------ complex

__host__ __device__ inline float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__host__ __device__ inline float2 cmulc(float2 a, float2 b) {  // conj(a) * b
  return make_float2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__host__ __device__ inline float2 cadd(float2 a, float2 b) {
  return make_float2(a.x + b.x, a.y + b.y);
}
__host__ __device__ inline float2 csub(float2 a, float2 b) {
  return make_float2(a.x - b.x, a.y - b.y);
}
__host__ __device__ inline float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
__host__ __device__ inline float2 cscale(float2 a, float s) {
  return make_float2(a.x * s, a.y * s);
}
__host__ __device__ inline float cabs2(float2 a) { return a.x * a.x + a.y * a.y; }

__host__ __device__ inline double2 zmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__host__ __device__ inline double2 zmulc(double2 a, double2 b) {  // conj(a) * b
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__host__ __device__ inline double2 zadd(double2 a, double2 b) {
  return make_double2(a.x + b.x, a.y + b.y);
}
__host__ __device__ inline double2 zsub(double2 a, double2 b) {
  return make_double2(a.x - b.x, a.y - b.y);
}
__host__ __device__ inline double2 zconj(double2 a) { return make_double2(a.x, -a.y); }
__host__ __device__ inline double2 zscale(double2 a, double s) {
  return make_double2(a.x * s, a.y * s);
}
__host__ __device__ inline double zabs2(double2 a) { return a.x * a.x + a.y * a.y; }

// ------------------------------------------------------------------ handle

struct TraceRec {
  const char* name;
  hipEvent_t begin, end;
};

struct Handle {
  hipStream_t stream = nullptr;
  uint32_t* status_dev = nullptr;   // device status word (PISCO_FLAG_*)
  uint32_t* host_pinned = nullptr;  // pinned host mirror for status/flags
  // fine-grained pinned words the schedule kernels write directly (host
  // pointer and the device's pointer to the same memory)
  int* host_ctl = nullptr;
  int* host_ctl_dev = nullptr;
  // recorded after the schedule kernel so that the host waits for it alone
  // while later work runs (created on first use by the adaptive schedule)
  hipEvent_t sched_ev = nullptr;
  std::string last_error;
  // kernel tracing (pisco_trace_enable): events bracket matching launches
  bool trace = false;
  std::string trace_filter;
  std::vector<hipEvent_t> event_pool;
  size_t events_used = 0;
  std::vector<TraceRec> records;
  // autotuner results per problem shape: nullspace block and product waves
  std::map<std::string, std::pair<int, int>> tuned;
  // plan-constant device tables (DFT and sinc matrices, support lists, index
  // maps) keyed by their exact parameters; freed by pisco_destroy.  A batch's
  // per-stream handles use their parent's (table_owner).
  std::map<std::string, void*> tables;
  Handle* table_owner = nullptr;
};

// A handle-owned device table of `bytes` bytes identified by `key`: on first
// use it is allocated, filled by `build` (kernels on the handle's stream)
// and the stream synchronised, so that any later stream may read it.  A
// first use while the stream is being captured is refused.
pisco_status_t cached_table(Handle* h, const std::string& key, size_t bytes, void** out,
                            const std::function<pisco_status_t(void*)>& build);

// Brackets one kernel launch with events when tracing is on and the kernel
// name contains the filter.
struct TraceScope {
  Handle* h;
  TraceRec rec{nullptr, nullptr, nullptr};
  TraceScope(Handle* hh, const char* name);
  ~TraceScope();
};

// Launch `kernel` on the handle's stream; traced when enabled; a launch error
// returns PISCO_ERR_HIP from the enclosing function.
#define PISCO_KERNEL(h, kernel, grid, block, shm, ...)                          \
  do {                                                                          \
    ::pisco::TraceScope pisco_ts_((h), #kernel);                                \
    hipLaunchKernelGGL(kernel, grid, block, shm, (h)->stream, __VA_ARGS__);     \
    hipError_t pisco_e_ = hipGetLastError();                                    \
    if (pisco_e_ != hipSuccess) return ::pisco::hip_check((h), pisco_e_, #kernel); \
  } while (0)

// ------------------------------------------------------------------ plan

constexpr int kMaxQ = 32;
constexpr int kAxSplit = 8;  // most K slices of the nullspace product A X
constexpr int kTnRows = 128;  // row chunk of the b x b products X^H Y
constexpr int kMaxSupport = 4096;

// Sizes derived from a problem description; everything a stage needs on the
// host to size launches and to lay out its workspace.
struct Plan {
  int D = 2, Q = 0;
  int acs[3] = {1, 1, 1};
  int tau = 0;            // floor(radius): half-width of the support box
  float radius = 0.f;
  int L = 0;              // |Lambda|
  int n = 0;              // Q |Lambda|
  int P = 0;              // Q (Q + 1) / 2 channel pairs
  int B[3] = {1, 1, 1};   // lag box extent per dim: 4 tau + 1 (1 for unused z)
  int nlag = 0;           // B0 * B1 * B2
  int F[3] = {1, 1, 1};   // FFT size per dim for the Gram correlation
  int nF = 0;
  int K[3] = {1, 1, 1};   // frequency grid of the filter correlations (= B)
  int nK = 0;
  int lr[3] = {1, 1, 1};
  int out[3] = {1, 1, 1};
  long long Nlr = 0, Nout = 0;
  float thresh = 0.05f;
};

// Fills `plan` from `prob`; returns PISCO_OK or an argument error with a
// message in `err`.
pisco_status_t make_plan(const pisco_problem_t* prob, Plan* plan, std::string* err);

// Enumerates the support in the library's order (host).
int enumerate_support(int D, float radius, int32_t* offsets /* 3 per point */,
                      int cap);

// ------------------------------------------------------------------ workspace carving

struct Carver {
  char* base;
  size_t used = 0;
  explicit Carver(void* b) : base(static_cast<char*>(b)) {}
  template <class T>
  T* take(size_t count) {
    size_t off = (used + 255) & ~size_t(255);
    used = off + count * sizeof(T);
    return reinterpret_cast<T*>(base ? base + off : nullptr);
  }
};

// Workspace layouts; each `layout_*` fills pointers when `ws` is non-null and
// returns the bytes used.
struct GramWs {
  float2* S;       // [Q][F0][F1][F2] coil spectra (plus the stage buffers)
  float2* T1;      // pair intermediates
  float2* T2;
  float2* R;       // [P][nlag] correlation lags
};
size_t layout_gram(const Plan& p, void* ws, GramWs* out);

struct NullWs {
  double2* X;      // [b][n] current orthonormal block (column-major n x b)
  double2* Z;      // [b][n] A X
  double2* H;      // [b][b] X^H Z
  double2* S;      // [b][b] Z^H Z
  double2* U;      // [b][b] Ritz vectors of H
  double2* M;      // [b][b] combined update
  double2* R;      // [b][b] Cholesky factor (column-major, upper)
  double* dsc;     // [b] column scaling of the factorised Gram
  double* theta;   // [b]
  double* filt;    // [12] Chebyshev filter coefficients: steps 1 and 2, the next product
  double* resid;   // [b]
  double2* part;   // row-chunk partials of the b x b products; residual partials
  int* ctl;        // [8] control words
  double* jac;     // Cholesky scratch (global-memory fallback) [b*(b+1)*2]
  double* heev;    // eigen-decomposition scratch [heev_workspace_doubles(b)]
};
size_t layout_null(const Plan& p, int b, void* ws, NullWs* out);

struct GxWs {
  float2* Fh;      // [b][Q][nK] filter spectra
  float2* Tmp;     // separable-transform scratch, two halves of tmp_half
  size_t tmp_half;
  float2* Kh;      // [P][nK] K^(f)
  float2* Klag;    // [P][nlag]
};
size_t layout_gx(const Plan& p, int b, void* ws, GxWs* out);

struct MapsWs {
  double2* rho;    // [Q][Nlr] apodized low-res images (FP64)
  double2* rtA;    // FP64 scratch of the apodized passes
  double2* rtB;
  double2* m;      // [Nlr] coil combination (FP64)
  double* pmax;    // per-block maxima of |m|
  float2* tmpA;    // separable-transform scratch
  float2* tmpB;
  float2* cref;    // [Q][Nlr] phase-referenced maps
};
size_t layout_maps(const Plan& p, void* ws, MapsWs* out);

// ------------------------------------------------------------------ stage launchers

pisco_status_t run_gram(Handle* h, const Plan& p, const float2* acs, float2* gram,
                        void* ws);
// fixed_products > 0: that many products and one Rayleigh-Ritz step, no host
// read-back (graph-capturable); 0: adaptive schedule with host reads.
// ax_waves: wave count targeted by the split-K product (0 = 2048).
// downstream (adaptive schedule only, nullable): enqueues the caller's later
// stages, which read basis/eigvals/counts; it is called after each
// Rayleigh-Ritz step before the host looks at the result (so that the GPU
// goes on while the host waits), again after a later step when that one was
// not final, and *downstream_queued tells the caller whether the last call
// stands.  Its work must not touch `ws`.
pisco_status_t run_nullspace(Handle* h, const Plan& p, int b, int max_iters,
                             const float2* gram, double* eigvals, double2* basis,
                             int32_t* counts, void* ws, int fixed_products = 0,
                             int ax_waves = 0,
                             const std::function<pisco_status_t()>* downstream = nullptr,
                             bool* downstream_queued = nullptr);
pisco_status_t run_gx(Handle* h, const Plan& p, int b, int precision, const double2* basis,
                      const int32_t* counts, float2* G, void* ws);
// lam64 / res64 (nullable): FP64 Rayleigh quotient and residual of the
// FP32 result, computed from the FP32 G widened to FP64.
pisco_status_t run_eig(Handle* h, int Q, long long N, float bound, int iters,
                       float tol, const float2* G, const float2* init, float2* maps,
                       float* lam, int32_t* it_out, double* lam64 = nullptr,
                       double* res64 = nullptr);
pisco_status_t run_maps(Handle* h, const Plan& p, int phase_rule, const float2* acs,
                        const float2* maps_lr, float2* maps_out, void* ws);

// The whole path for one problem on h's stream (pisco_estimate's body);
// fixed_products / ax_waves as for run_nullspace; counts_out (nullable)
// receives the device address of the nullspace counts in `ws`.
size_t estimate_ws_size(const Plan& p, int b);
pisco_status_t estimate_core(Handle* h, const Plan& p, const pisco_opts_t& o, int b,
                             const float2* acs, float2* maps_out, float* lam_min, void* ws,
                             int fixed_products, int ax_waves, int32_t** counts_out = nullptr);

// Eigen-decomposition H = U diag(theta) U^H of a b x b Hermitian matrix
// (column-major, FP64), eigenvalues descending, 1 <= b <= 1024; `ws` holds
// heev_workspace_doubles(b) doubles (device).
size_t heev_workspace_doubles(int b);
pisco_status_t run_heev(Handle* h, const double2* H, int b, double2* U, double* theta,
                        double* ws);

// Separable transform along one axis of a batched 3D array:
//   out[b][..o..] = sum_i M[o][i] * in[b][..i..]
// shape_in = {batch, d0, d1, d2}; axis in {1,2,3}; M is [nout][nin] float2.
pisco_status_t axis_transform(Handle* h, const float2* in, float2* out,
                              const int shape_in[4], int axis, int nout,
                              const float2* M);

// Matrix builders (float2, row-major [nout][nin]) for axis_transform:
//   build_dft : M[o][i] = scale * g(i) * exp(i sign 2 pi (i - ci)(o - co) / period),
//               g(i) = exp(-(i - ci)^2 / (2 sigma^2)) if sigma > 0 else 1
//   build_sinc: periodic sinc interpolation n_in -> n_out centred samples
pisco_status_t build_dft(Handle* h, float2* M, int nout, int nin, int co, int ci,
                         double period, double sign, double scale, double sigma);
pisco_status_t build_dft(Handle* h, double2* M, int nout, int nin, int co, int ci,
                         double period, double sign, double scale, double sigma);
// FP64 variants of axis_transform (input FP32 or FP64, output and matrix FP64)
pisco_status_t axis_transform64(Handle* h, const float2* in, double2* out,
                                const int shape_in[4], int axis, int nout, const double2* M);
pisco_status_t axis_transform64(Handle* h, const double2* in, double2* out,
                                const int shape_in[4], int axis, int nout, const double2* M);
pisco_status_t build_sinc(Handle* h, float2* M, int nout, int nin);

// Writes the support offsets (z, y, x, 0) into `out` on the device.
// Handle-cached (plan-constant) tables: the builders above and the support
// list of |Lambda| = L points (cached_table); valid until pisco_destroy.
pisco_status_t dft_table(Handle* h, const float2** M, int nout, int nin, int co, int ci,
                         double period, double sign, double scale, double sigma);
pisco_status_t dft_table(Handle* h, const double2** M, int nout, int nin, int co, int ci,
                         double period, double sign, double scale, double sigma);
pisco_status_t sinc_table(Handle* h, const float2** M, int nout, int nin);
pisco_status_t support_table(Handle* h, const int4** out, int D, float radius, int L);

inline pisco_status_t hip_check(Handle* h, hipError_t e, const char* what) {
  if (e == hipSuccess) return PISCO_OK;
  if (h) h->last_error = std::string(what) + ": " + hipGetErrorString(e);
  return PISCO_ERR_HIP;
}

#define PISCO_LAUNCH_CHECK(h, what)                                   \
  do {                                                                \
    hipError_t e_ = hipGetLastError();                                \
    if (e_ != hipSuccess) return ::pisco::hip_check((h), e_, (what)); \
  } while (0)

inline unsigned ceil_div(long long a, long long b) { return unsigned((a + b - 1) / b); }

}  // namespace pisco
