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

// Orders the LDS accesses of one wave around it, for kernels whose
// workgroup is a single wave (a wave's LDS operations are performed in
// order): no s_barrier and no wait on memory counters.
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Workgroup b of nb is dispatched to XCD b % 8 (each XCD has its own L2);
// the logical index gives each XCD a contiguous range of [0, nb) (a
// bijection), so that neighbouring logical workgroups share one L2.
constexpr int kXcds = 8;
__device__ inline long long xcd_block(unsigned b, unsigned nb) {
  const unsigned x = b % kXcds, k = b / kXcds, q = nb / kXcds, r = nb % kXcds;
  const unsigned base = x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q;
  return (long long)base + k;
}

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
  // compute units of the device current at creation (persistent grids)
  int num_cu = 256;
};

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
  int shape = PISCO_SHAPE_ELLIPSOID;  // support shape
  int rows = PISCO_ROWS_ALL;          // rows of C in the Gram
  long long Pvalid = 0;               // rows of C_valid: prod (A_d - 2 tau)
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
int enumerate_support(int D, float radius, int shape, int32_t* offsets /* 3 per point */,
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
  float2* C;       // [Pvalid][n] rows of C_valid (PISCO_ROWS_VALID only)
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
  int* ctl;        // [16] control words, then the device-resident schedule
  double* jac;     // Cholesky scratch (global-memory fallback) [b*(b+1)*2]
  double* heev;    // eigen-decomposition scratch [heev_workspace_doubles(b)]
  // structured products only (null otherwise): per-frequency Gram blocks
  // [F^D + 1][kMaxQ][kMaxQ] and two spectrum buffers of toeplitz_spectrum_elems each
  double2* rhat;
  double2* sp0;
  double2* sp1;
};
size_t layout_null(const Plan& p, int b, void* ws, NullWs* out, bool structured = false);

// Gram products through the correlation structure (toeplitz.hip): the lags
// R_pq[d] on the (4 tau + 1)^D box stand for the Gram.
struct ToeplitzOp {
  const float2* lags;   // [P][Bz][B][B] (Bz = 1 when D = 2), as the Gram stage forms them
  const int* boxmap;    // [Wz][W][W] box cell -> support index, -1 outside
  const int4* sup;      // support points (z, y, x, 0)
  const double2* Tf;    // F x W: box -> frequency
  const double2* Ti;    // W x F: frequency -> box, 1/F included
  const double2* Tr;    // F x F: lags -> frequency
  double2* rhat;        // [Fz F F + 1][kMaxQ][kMaxQ], toeplitz_rhat_elems
  double2* buf0;        // spectrum buffers, toeplitz_spectrum_elems(p, b) each
  double2* buf1;
  int D, W, Wz, F, Fz, Q, L, P;
};
size_t toeplitz_spectrum_elems(const Plan& p, int b);
size_t toeplitz_rhat_elems(const Plan& p);
// rhat from the lags (once per nullspace call; uses buf0 / buf1).
pisco_status_t toeplitz_prepare(Handle* h, const ToeplitzOp& op);
// out = A X (or the Chebyshev step / role of the explicit product) for a
// column-major n x b block.
pisco_status_t toeplitz_product(Handle* h, const ToeplitzOp& op, const double2* X,
                                double2* out, int n, int b, const double* coef,
                                const double2* prev, const int* role);

struct GxWs {
  float2* Fh;      // [b][Q][nK] filter spectra
  float2* Tmp;     // separable-transform scratch, two halves of tmp_half
  size_t tmp_half;
  float2* Kh;      // [P][nK] K^(f)
};
size_t layout_gx(const Plan& p, int b, void* ws, GxWs* out);

// Plan-constant tables (functions of the sizes alone), carved from the
// caller's workspace and built by one kernel in stream order by the call
// that uses them, so that no call allocates or synchronises.
//   sup    : int4 [L], support offsets (z, y, x, 0) in the library's order
//   boxmap : int [box^D], support-box cell -> support index (-1 outside)
//   M1[d]  : float2 [K_d][2 tau + 1]  filter spectra  e^{+i 2 pi n f / K_d}
//   M4[d]  : float2 [lr_d][K_d]       low-res evaluation from the spectra: the lags
//                                     (1/K_d) e^{+i 2 pi m f / K_d}, |m| <= 2 tau,
//                                     evaluated at e^{-i 2 pi m x} and summed (FP64)
//   Ma[d]  : double2 [lr_d][A_d]      apodized low-res image (FP64)
//   Ms[d]  : float2 [out_d][lr_d]     periodic sinc interpolation
//   Ms64[d]: double2 [out_d][lr_d]    the same in FP64 (support mask)
// Dimensions d that the problem does not use (z for D = 2) stay null.
struct Tables {
  int4* sup = nullptr;
  int* boxmap = nullptr;
  float2* M1[3] = {nullptr, nullptr, nullptr};
  float2* M4[3] = {nullptr, nullptr, nullptr};
  double2* Ma[3] = {nullptr, nullptr, nullptr};
  float2* Ms[3] = {nullptr, nullptr, nullptr};
  double2* Ms64[3] = {nullptr, nullptr, nullptr};
  double2* Tf = nullptr;  // structured products: box -> frequency (F x W)
  double2* Ti = nullptr;  // frequency -> box (W x F, 1/F included)
  double2* Tr = nullptr;  // lags -> frequency (F x F)
};
// Which tables a call needs (bit mask).
constexpr unsigned kTabSupport = 1u, kTabGx = 2u, kTabMaps = 4u, kTabMask = 8u,
                   kTabToeplitz = 16u;
constexpr unsigned kTabAll = kTabSupport | kTabGx | kTabMaps | kTabToeplitz;
// Carves the tables of `which` from `ws` (sizes only when ws is null);
// returns the bytes used.
size_t layout_tables(const Plan& p, unsigned which, void* ws, Tables* out);
// Builds the tables of `which` (one kernel launch).
pisco_status_t build_tables(Handle* h, const Plan& p, unsigned which, const Tables& t);

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
// order of the interpolation passes over the used axes (0 = z, 1 = y, 2 = x):
// x last, z and y ascending in out / lr; returns the number of used axes (D)
int interp_order(const Plan& p, int ord[3]);

// ------------------------------------------------------------------ stage launchers

// support_ws (nullable): region of L int4 where the support list is built in
// stream order instead of taken from the handle's table.
// lags_out (nullable): the lags R_pq go there ([P][nlag]) and the Gram is
// not gathered (gram unused).
pisco_status_t run_gram(Handle* h, const Plan& p, const Tables& t, const float2* acs,
                        float2* gram, void* ws, float2* lags_out = nullptr);
// The Gram with the library's static per-device scratch (kGramScratchBytes)
// as workspace: no allocation; calls that overlap on one GPU race.
constexpr size_t kGramScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;
size_t gram_static_bytes(const Plan& p);
pisco_status_t run_gram_static(Handle* h, const Plan& p, const float2* acs, float2* gram);
// Per-device address of that scratch (resolved once per device).
pisco_status_t gram_scratch_address(Handle* h, void** out);
// fixed_products > 0: that many products and one Rayleigh-Ritz step, no host
// read-back (graph-capturable); 0: adaptive schedule with host reads.
// ax_waves: wave count targeted by the split-K product (0 = 2048).
// downstream (adaptive schedule only, nullable): enqueues the caller's later
// stages, which read basis/eigvals/counts; it is called after each
// Rayleigh-Ritz step before the host looks at the result (so that the GPU
// goes on while the host waits), again after a later step when that one was
// not final, and *downstream_queued tells the caller whether the last call
// stands.  Its work must not touch `ws`.
// tp (nullable): products through the correlation structure (gram unused;
// ws laid out with layout_null(..., structured = true)).
pisco_status_t run_nullspace(Handle* h, const Plan& p, int b, int max_iters,
                             const float2* gram, double* eigvals, double2* basis,
                             int32_t* counts, void* ws, int fixed_products = 0,
                             int ax_waves = 0,
                             const std::function<pisco_status_t()>* downstream = nullptr,
                             bool* downstream_queued = nullptr, int device_products = 0,
                             const ToeplitzOp* tp = nullptr);
// Products the device-resident schedule enqueues (the cap on the products
// it can run): at most kDeviceProducts, fewer when max_iters is smaller.
constexpr int kDeviceProducts = 16;
// Schedule of a nullspace call: device_products for run_nullspace (0 =
// adaptive host-read schedule), or an error when that schedule is refused.
pisco_status_t choose_schedule(Handle* h, const pisco_opts_t& o, int* device_products);
pisco_status_t run_gx(Handle* h, const Plan& p, const Tables& t, int b, int precision,
                      const double2* basis, const int32_t* counts, float2* G, void* ws);
// lam64 / res64 (nullable): FP64 Rayleigh quotient and residual of the
// FP32 result, computed from the FP32 G widened to FP64.
pisco_status_t run_eig(Handle* h, int Q, long long N, float bound, int iters,
                       float tol, const float2* G, const float2* init, float2* maps,
                       float* lam, int32_t* it_out, double* lam64 = nullptr,
                       double* res64 = nullptr);
pisco_status_t run_maps(Handle* h, const Plan& p, const Tables& t, int phase_rule,
                        const float2* acs, const float2* maps_lr, float2* maps_out, void* ws);

// The M smallest eigenpairs per voxel by K Lanczos steps (1 <= M <= 8,
// M <= K <= Q): maps [M][Q][N], lam [M][N], resid [M][N] (nullable).
// run_eig_sets takes G entry-major ([Q(Q+1)/2][N], as from the G(x) stage)
// and copies it voxel-major into ws (layout_eig_sets bytes);
// run_lanczos_vm takes G voxel-major ([N][Q(Q+1)/2]) directly.
size_t layout_eig_sets(int Q, long long N);
pisco_status_t run_eig_sets(Handle* h, int Q, long long N, float bound, int K, int M,
                            const float2* G, float2* maps, float* lam, float* resid, void* ws);
pisco_status_t run_lanczos_vm(Handle* h, int Q, long long N, float bound, int K, int M,
                              const float2* Gvm, float2* maps, float* lam, float* resid);

// Partial SVDs of B Casorati matrices X [B][Q][m] (r <= min(8, Q)): sigma
// [r][B], right singular vectors [r][Q][B] (Vout nullable: in ws), rank-r
// part Xr [B][Q][m] (nullable).
size_t layout_llr(long long B, int Q, int r, void* ws, float2** A, float2** V, float** lam);
pisco_status_t run_llr(Handle* h, long long B, int m, int Q, int r, const float2* X,
                       float* sigma, float2* Vout, float2* Xr, void* ws);

// Support mask (FP64 interpolation of lambda_min / bound, thresholded) and
// the ESPIRiT operator B = I - G / bound on packed planes.
size_t layout_mask(const Plan& p, void* ws, double2** t0, double2** t1, double2** t2);
pisco_status_t run_support_mask(Handle* h, const Plan& p, const Tables& t, const float* lam,
                                float bound, float thresh, uint8_t* mask, void* ws);
pisco_status_t run_espirit_operator(Handle* h, int Q, long long N, float bound,
                                    const float2* G, float2* B);

// The whole path for one problem on h's stream (pisco_estimate's body);
// fixed_products / ax_waves as for run_nullspace; counts_out (nullable)
// receives the device address of the nullspace counts in `ws`.
// structured: Gram products through the correlation structure (the Gram is
// not formed; see structured_product).
size_t estimate_ws_size(const Plan& p, int b, bool structured);
bool structured_product(const Plan& p, const pisco_opts_t& o);
// tables_ready: the tables in `ws` were built by an earlier run with the
// same problem and block (a batch's captured graph skips rebuilding them).
pisco_status_t estimate_core(Handle* h, const Plan& p, const pisco_opts_t& o, int b,
                             const float2* acs, float2* maps_out, float* lam_min, void* ws,
                             int fixed_products, int ax_waves, int32_t** counts_out = nullptr,
                             bool tables_ready = false);

// Eigen-decomposition H = U diag(theta) U^H of a b x b Hermitian matrix
// (column-major, FP64), eigenvalues descending, 1 <= b <= 1024; `ws` holds
// heev_workspace_doubles(b) doubles (device).
size_t heev_workspace_doubles(int b);
pisco_status_t run_heev(Handle* h, const double2* H, int b, double2* U, double* theta,
                        double* ws);

// Separable transform along one axis of a batched 3D array:
//   out[b][..o..] = sum_i M[o][i] * in[b][..i..]
// shape_in = {batch, d0, d1, d2}; axis in {1,2,3}; M is [nout][nin] float2.
// real_m: M's imaginary parts are zero and may be skipped (sinc tables).
pisco_status_t axis_transform(Handle* h, const float2* in, float2* out,
                              const int shape_in[4], int axis, int nout,
                              const float2* M, bool real_m = false);

// Last interpolation pass along x with a real M ([nout][nin], imaginary
// parts ignored) fused with the per-voxel coil normalisation:
//   out[q][r][o] = y[q][r][o] / ||y[:, r, o]||_2,  y[q][r][o] = sum_i M[o][i] in[q][r][i]
// (a zero norm leaves y).  PISCO_ERR_UNSUPPORTED when the shape does not fit
// (Q > 64 or nin > 64); nothing is launched then.
pisco_status_t interp_x_rss(Handle* h, const float2* in, float2* out, const float2* M, int Q,
                            long long rows, int nin, int nout);

// axis_transform whose outer index is the packed Hermitian pair of a Q x Q
// matrix, stored as G = bound I - y (diagonal pairs real).  Only on the
// matrix-core column path; PISCO_ERR_UNSUPPORTED (nothing launched) otherwise.
pisco_status_t axis_transform_gx(Handle* h, const float2* in, float2* out,
                                 const int shape_in[4], int axis, int nout, const float2* M,
                                 int Q, float bound);

// FP64 variants of axis_transform (input FP32 or FP64, output and matrix FP64)
pisco_status_t axis_transform64(Handle* h, const float2* in, double2* out,
                                const int shape_in[4], int axis, int nout, const double2* M);
pisco_status_t axis_transform64(Handle* h, const double2* in, double2* out,
                                const int shape_in[4], int axis, int nout, const double2* M);


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
