/*
 * pisco.h -- C ABI of the MI355X (gfx950) implementation of PISCO subspace
 * sensitivity-map estimation (Lobos, Chan, Haldar: "New Theory and Faster
 * Computations for Subspace-Based Sensitivity Map Estimation in Multichannel
 * MRI", extended version).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - All array arguments except those marked "host" are DEVICE pointers owned
 *    by the caller.  Scratch space comes from the caller's workspace, whose
 *    size is given by pisco_workspace_size().  Workspace pointers must be
 *    256-byte aligned.  No call allocates device memory: the plan-constant
 *    tables (DFT and sinc matrices, the support list and its box map, a
 *    function of the sizes alone) live at the front of the workspace and
 *    are rebuilt by one small kernel at the start of every call that uses
 *    them.
 *  - Calls enqueue kernels on the handle's stream and return without
 *    synchronising, except where stated (pisco_get_status, pisco_trace_read,
 *    pisco_batch_create, and the adaptive schedule of pisco_nullspace /
 *    pisco_estimate, which waits on events for its control words).  Results
 *    are valid once the stream has been synchronised.  No call issues
 *    hipMemsetAsync or host<->device copies, so calls other than the
 *    adaptive schedule can be captured into a HIP graph.
 *  - Complex data are interleaved single-precision pairs (float2, re then im)
 *    unless marked double2.
 *  - Spatial arrays are stored [z][y][x] with x fastest.  For D = 2 the z
 *    extent is 1.  Along a dimension of length L, index a corresponds to the
 *    integer frequency k = a - floor(L/2) (k-space) and to the position
 *    x = (a - floor(L/2)) / L (image space), i.e. the field of view is
 *    [-1/2, 1/2)^D with unit k-space spacing (Sec. III-A, Eqs. 2-4).
 *  - The kernel support Lambda = { n in Z^D : ||n||_2 <= radius } (Sec. IV-B)
 *    is ordered lexicographically, z slowest and x fastest; |Lambda| is
 *    returned by pisco_support().  n = Q |Lambda| is the Gram dimension and
 *    filter vectors are indexed q |Lambda| + i (the column order of
 *    C = [C_1 ... C_Q], Eq. 14).
 *  - Return codes: PISCO_OK, or an error detected on the host before any
 *    launch (bad argument, workspace too small, unsupported size) or reported
 *    by the HIP runtime on launch.  Numerical conditions found on the device
 *    (non-finite input, nullspace iteration not converged) are recorded in
 *    the handle's device status word and read with pisco_get_status().
 *    pisco_last_error() gives a message for the last failing call.
 *  - No C++ exception or abort crosses this interface.
 */
#ifndef PISCO_H
#define PISCO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PISCO_OK = 0,
  PISCO_ERR_ARG = 1,         /* invalid argument (null pointer, bad size) */
  PISCO_ERR_WORKSPACE = 2,   /* workspace smaller than pisco_workspace_size */
  PISCO_ERR_HIP = 3,         /* HIP runtime error (launch, device) */
  PISCO_ERR_UNSUPPORTED = 4, /* size outside what the kernels support */
  PISCO_ERR_NUMERIC = 5      /* numeric failure reported by the device */
} pisco_status_t;

/* Device status flags (bits of the word returned by pisco_get_status). */
#define PISCO_FLAG_NONFINITE      0x1u  /* NaN/Inf met in an input or result */
#define PISCO_FLAG_NOT_CONVERGED  0x2u  /* nullspace iteration hit its cap    */
#define PISCO_FLAG_BLOCK_TOO_SMALL 0x4u /* signal rank reached the block size */
#define PISCO_FLAG_ZERO_DATA      0x8u  /* all-zero calibration data          */

typedef struct pisco_handle_s* pisco_handle_t;

/* Problem description (Sec. III-A, IV-B, IV-D). */
typedef struct {
  int32_t D;            /* 2 or 3 */
  int32_t Q;            /* number of channels, 2..32 */
  int32_t acs[3];       /* calibration (ACS) extent z, y, x; acs[0] = 1 for D = 2 */
  float radius;         /* kernel radius tau of the ellipsoidal support (Sec. IV-B) */
  int32_t grid_lr[3];   /* low-resolution estimation grid z, y, x (Sec. IV-D) */
  int32_t grid_out[3];  /* output grid z, y, x; each >= grid_lr */
  float thresh;         /* nullspace rule sigma_n < thresh * sigma_1; 0.05 in the
                           paper (Sec. III-B footnote) */
  int32_t shape;        /* kernel support: PISCO_SHAPE_ELLIPSOID (Sec. IV-B) or
                           PISCO_SHAPE_RECTANGLE (the conventional support of
                           Sec. III-C) */
  int32_t gram_rows;    /* rows of C in the Gram: PISCO_ROWS_ALL (every row
                           the data touch, samples outside the ACS taken as
                           zero: the correlation form of Sec. IV-A) or
                           PISCO_ROWS_VALID (only rows whose whole
                           neighbourhood lies inside the ACS: no implicit
                           zeros, the masked form Sec. IV-A neglects) */
} pisco_problem_t;

/* Support shapes (pisco_problem_t.shape). */
#define PISCO_SHAPE_ELLIPSOID 0  /* { n : ||n||_2 <= radius } */
#define PISCO_SHAPE_RECTANGLE 1  /* { n : ||n||_inf <= floor(radius) } */

/* Gram rows (pisco_problem_t.gram_rows). */
#define PISCO_ROWS_ALL   0
#define PISCO_ROWS_VALID 1

/* Options of the per-voxel solve and the nullspace iteration. */
typedef struct {
  int32_t power_iters;  /* power-iteration steps (10 in the paper, Sec. IV-E);
                           in tolerance mode the cap on steps */
  float tol;            /* 0: fixed step count; > 0: stop a voxel once
                           ||G c - lambda c||_2 <= tol * |Lambda| */
  int32_t phase_rule;   /* 0: cancel the phase of the coil-combined apodized
                           low-resolution image (Sec. IV-D); 1: reference to
                           channel 0 (Sec. V) */
  int32_t block;        /* nullspace block size (multiple of 32, 0 = automatic) */
  int32_t max_subspace_iters; /* cap on nullspace iterations (0 = 60) */
  int32_t precision;    /* arithmetic of the G(x) contraction over the signal
                           vectors: PISCO_PREC_FP32, or matrix cores with FP32
                           accumulation and split operands (PISCO_PREC_SPLIT_*) */
  int32_t schedule;     /* nullspace schedule: PISCO_SCHED_AUTO or
                           PISCO_SCHED_DEVICE (see pisco_nullspace) */
  int32_t product;      /* Gram products of pisco_estimate's nullspace:
                           PISCO_PRODUCT_AUTO, _DENSE or _STRUCTURED */
} pisco_opts_t;

/* Gram products in pisco_estimate (pisco_opts_t.product).  DENSE forms the
 * n x n Gram and multiplies it on the FP64 matrix cores.  STRUCTURED never
 * forms it: Gram[(p,i),(q,j)] = R_pq[n_i - n_j] (Sec. IV-A), so A X is a sum
 * of correlations of each column with the lags, evaluated exactly (FP64) on
 * the (4 tau + 1)^D frequency grid: pruned DFT passes and one Q x Q product
 * per frequency, 8 (4 tau + 1)^D Q^2 b flops against 8 n^2 b.  AUTO picks
 * STRUCTURED for 3D problems with n >= 4096 and the correlation Gram (gram_rows
 * = PISCO_ROWS_ALL), DENSE otherwise.  pisco_nullspace always takes the
 * explicit Gram. */
#define PISCO_PRODUCT_AUTO       0
#define PISCO_PRODUCT_DENSE      1
#define PISCO_PRODUCT_STRUCTURED 2

/* Nullspace schedules (pisco_opts_t.schedule). */
#define PISCO_SCHED_AUTO   0  /* adaptive (host reads control words) outside
                                 stream capture, device-resident under capture */
#define PISCO_SCHED_DEVICE 1  /* device-resident: never reads back on the host */

/* Precision choices (pisco_opts_t.precision). */
#define PISCO_PREC_FP32       0  /* FP32 arithmetic */
#define PISCO_PREC_SPLIT_F16  1  /* FP16 MFMA, each operand as 2 FP16 parts,
                                    3 cross products, FP32 accumulation */
#define PISCO_PREC_SPLIT_BF16 2  /* BF16 MFMA, each operand as 3 BF16 parts,
                                    6 cross products, FP32 accumulation */

/* Stage identifiers for pisco_workspace_size. */
#define PISCO_STAGE_GRAM      1
#define PISCO_STAGE_NULLSPACE 2
#define PISCO_STAGE_GX        3
#define PISCO_STAGE_EIG       4
#define PISCO_STAGE_MAPS      5
#define PISCO_STAGE_MASK      6   /* pisco_support_mask */
#define PISCO_STAGE_ALL       0   /* pisco_estimate, intermediates included */

/* Handle creation.  `stream` is a hipStream_t (NULL = default stream).  The
 * handle owns host state, one small device status word and a few pinned
 * host control words, all allocated here and freed by pisco_destroy.  It
 * also resolves, for the current device, the address of the static scratch
 * that pisco_gram_static uses.  A handle must not be used from two threads
 * at once. */
pisco_status_t pisco_create(pisco_handle_t* handle, void* stream);
pisco_status_t pisco_destroy(pisco_handle_t handle);
pisco_status_t pisco_set_stream(pisco_handle_t handle, void* stream);
const char* pisco_status_string(pisco_status_t status);
const char* pisco_last_error(pisco_handle_t handle);

/* Synchronises the handle's stream, then returns the device status flags
 * accumulated since the last call and clears them (host pointer `flags`). */
pisco_status_t pisco_get_status(pisco_handle_t handle, uint32_t* flags);

/* Kernel support (Sec. IV-B; shape PISCO_SHAPE_*).  Host-only.  Writes
 * |Lambda| to *count and, when `offsets` (host, int32[3 * count], z y x per
 * point) is non-null, the offsets in the library's order.  Needs D in {2,3},
 * radius in [1, 12]. */
pisco_status_t pisco_support(int32_t D, float radius, int32_t shape, int32_t* count,
                             int32_t* offsets);

/* Bytes of workspace needed by one stage (or by pisco_estimate when stage is
 * PISCO_STAGE_ALL).  `opts` may be NULL (defaults).  Host-only. */
pisco_status_t pisco_workspace_size(const pisco_problem_t* prob,
                                    const pisco_opts_t* opts, int32_t stage,
                                    size_t* bytes);

/* Calibration Gram C^H C.  With PISCO_ROWS_ALL by zero-padded FFT
 * correlation (Sec. IV-A), as below; with PISCO_ROWS_VALID the rows of C
 * whose neighbourhood n - Lambda lies inside the ACS (a box of
 * prod_d (A_d - 2 floor(radius)) rows) are formed explicitly and C^H C is
 * their FP32 product (the masked Gram, exactly Hermitian as well). */
/* Calibration Gram C^H C by zero-padded FFT correlation (Sec. IV-A).
 *   acs  : float2 [Q][acs z][acs y][acs x], the Nyquist-sampled ACS block
 *   gram : float2 [n][n], n = Q |Lambda|, row-major; entry ((p,i),(q,j)) is
 *          R_pq[n_i - n_j] with R_pq[d] = sum_k conj(s_p[k]) s_q[k+d]
 *          (samples outside the ACS are zero: the unmasked form the paper
 *          uses, equal to C^H C over every row the data touch).  Exactly
 *          Hermitian (the lower triangle is written as the conjugate of the
 *          upper). */
pisco_status_t pisco_gram(pisco_handle_t handle, const pisco_problem_t* prob,
                          const void* acs, void* gram, void* workspace,
                          size_t workspace_bytes);

/* pisco_gram for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * the same kernels and results as pisco_gram, with no workspace argument.
 * Scratch comes from a library-owned static device array of
 * pisco_gram_static_bytes' `limit` bytes (64 MiB), one per GPU, held until
 * the process ends; its address is resolved at pisco_create (or at the first
 * call on another device).  The call allocates nothing and builds no handle
 * table (the support list is rebuilt in the scratch on every call).
 * Problems whose scratch need exceeds the limit are rejected with
 * PISCO_ERR_UNSUPPORTED before any launch.  Every call on a GPU shares that
 * GPU's array: calls that may overlap on one GPU (other streams, other
 * handles, other threads) race and must be serialised by the caller. */
pisco_status_t pisco_gram_static(pisco_handle_t handle, const pisco_problem_t* prob,
                                 const void* acs, void* gram);

/* Scratch bytes pisco_gram_static needs for `prob`, and the library's limit
 * (either pointer may be NULL).  Host-only. */
pisco_status_t pisco_gram_static_bytes(const pisco_problem_t* prob, size_t* bytes,
                                       size_t* limit);

/* Signal/null split of the Gram (Sec. III-A/B; threshold from the footnote
 * of Sec. III-B).  FP64 block subspace iteration with Rayleigh-Ritz on the
 * FP32 Gram widened exactly to FP64.  The filters h_r of the paper are the
 * eigenvectors with lambda < thresh^2 lambda_1; their complement, the signal
 * eigenvectors, is returned because the nullspace projector is
 * I - V_s V_s^H (the route of Eq. 20).
 *   gram    : float2 [n][n] from pisco_gram (only the Hermitian part is used)
 *   eigvals : double [block], Ritz values, descending; the first counts[0]
 *             are the signal eigenvalues lambda_k >= thresh^2 lambda_1
 *   basis   : double2 [block][n], Ritz vectors, one contiguous vector per
 *             row, orthonormal; the first counts[0] span the signal space
 *   counts  : int32 [4] written on the device: {r_signal, block,
 *             iterations used, 1 if converged else 0}
 * `block` is opts->block or the automatic size (pisco_nullspace_block).
 *
 * Schedule.  After three products (each orthonormalised) the Cholesky
 * diagonal predicts how many more products the Rayleigh-Ritz step needs and
 * sets the Chebyshev filter of the later chains.
 *  - Adaptive (PISCO_SCHED_AUTO outside capture): the host waits on events
 *    for that prediction and for the result of each Rayleigh-Ritz step (a
 *    step that does not converge schedules more products).  This call then
 *    blocks until those control words are written; it cannot be captured.
 *  - Device-resident (PISCO_SCHED_DEVICE, or AUTO while the stream is being
 *    captured): min(16, max_subspace_iters) products are enqueued in fixed
 *    chains with one Rayleigh-Ritz step after the last; the device turns the
 *    leading surplus products into block copies, so the step follows as many
 *    products as predicted.  Nothing is read back; a result that has not
 *    converged by the last product raises PISCO_FLAG_NOT_CONVERGED. */
pisco_status_t pisco_nullspace(pisco_handle_t handle,
                               const pisco_problem_t* prob,
                               const pisco_opts_t* opts, const void* gram,
                               double* eigvals, void* basis, int32_t* counts,
                               void* workspace, size_t workspace_bytes);

/* Block size pisco_nullspace uses for this problem (host-only). */
pisco_status_t pisco_nullspace_block(const pisco_problem_t* prob,
                                     const pisco_opts_t* opts, int32_t* block);

/* Per-voxel G(x) = H(x)^H H(x) on the low-resolution grid (Sec. IV-C,
 * Eqs. 23-26), from the lag sums of the nullspace filters' correlations.
 *   basis, counts : outputs of pisco_nullspace (counts read on the device)
 *   G : float2 [Q(Q+1)/2][N_lr], packed upper triangle, entry (p,q) with
 *       p <= q at index p*Q - p*(p-1)/2 + (q - p); each entry is a
 *       contiguous plane over the voxels of grid_lr. */
pisco_status_t pisco_gx(pisco_handle_t handle, const pisco_problem_t* prob,
                        const pisco_opts_t* opts, const void* basis,
                        const int32_t* counts, void* G, void* workspace,
                        size_t workspace_bytes);

/* Per-voxel eigenvector of G(x) for its smallest eigenvalue by power
 * iteration on |Lambda| I - G(x) (Sec. III-D step 4, Sec. IV-E).  The start
 * vector is e_q with q the smallest diagonal entry of G(x) (lowest index on
 * ties).
 *   G        : float2 packed as produced by pisco_gx, N voxels
 *   bound    : |Lambda| (the spectrum of G lies in [0, bound])
 *   maps     : float2 [Q][N], unit-norm eigenvector per voxel
 *   lam_min  : float [N], c^H G c (may be NULL)
 *   iters    : int32 [N], steps taken (may be NULL) */
pisco_status_t pisco_eig(pisco_handle_t handle, int32_t Q, int64_t N,
                         float bound, const pisco_opts_t* opts, const void* G,
                         void* maps, float* lam_min, int32_t* iters,
                         void* workspace, size_t workspace_bytes);

/* Phase reference, periodic sinc interpolation and sum-of-squares
 * normalisation (Sec. IV-D, Sec. V).
 *   acs      : float2 [Q][acs], used for the apodized low-resolution image
 *   maps_lr  : float2 [Q][grid_lr] from pisco_eig
 *   maps_out : float2 [Q][grid_out], unit root-sum-of-squares per voxel */
pisco_status_t pisco_maps(pisco_handle_t handle, const pisco_problem_t* prob,
                          const pisco_opts_t* opts, const void* acs,
                          const void* maps_lr, void* maps_out, void* workspace,
                          size_t workspace_bytes);

/* As pisco_eig, starting each voxel from the caller's vector instead of e_q
 * (a warm start, e.g. from pisco_ws_forward).
 *   init : float2 [Q][N]; normalised here; a voxel whose start vector is zero
 *          or not finite falls back to e_q. */
pisco_status_t pisco_eig_from(pisco_handle_t handle, int32_t Q, int64_t N,
                              float bound, const pisco_opts_t* opts,
                              const void* G, const void* init, void* maps,
                              float* lam_min, int32_t* iters, void* workspace,
                              size_t workspace_bytes);

/* As pisco_eig_from (init may be NULL: start from e_q*), plus an FP64
 * Rayleigh check of the FP32 result (Sec. IV-E; the final check the method
 * keeps in FP64): with c the stored map widened to FP64 and normalised, and
 * G the FP32 input widened exactly,
 *   lam64   : double [N], c^H G c (may be NULL)
 *   resid64 : double [N], ||G c - lam64 c||_2 (may be NULL). */
pisco_status_t pisco_eig_checked(pisco_handle_t handle, int32_t Q, int64_t N,
                                 float bound, const pisco_opts_t* opts,
                                 const void* G, const void* init, void* maps,
                                 float* lam_min, int32_t* iters, double* lam64,
                                 double* resid64, void* workspace,
                                 size_t workspace_bytes);

/* The `sets` smallest eigenpairs of G(x) per voxel by `krylov` Lanczos
 * steps (Sec. IV-E: the remedy the paper names where the two smallest
 * singular values are close and power iteration is slow; Sec. III-B
 * footnote: one set of maps per small eigenvalue when the field of view is
 * too small).  Lanczos on G(x) from e_q* (three-term recurrence and one
 * full reorthogonalisation pass per step; restarts from the least covered
 * coordinate after an invariant subspace), the
 * tridiagonal projection solved in FP64, Ritz vectors of the smallest Ritz
 * values; with krylov = Q the pairs are G's own to FP32 rounding.
 *   G     : float2 packed as from pisco_gx, N voxels
 *   bound : |Lambda| (scale of the invariant-subspace test); a value <= 0
 *           uses each voxel's largest row sum of |G| instead
 *   sets  : 1..min(8, krylov);  krylov : 1..Q
 *   maps  : float2 [sets][Q][N], unit-norm eigenvectors, ascending eigenvalue
 *   lam   : float [sets][N], Rayleigh quotients c^H G c
 *   resid : float [sets][N], ||G c - lam c|| (may be NULL)
 * Workspace: pisco_eig_sets_workspace_size bytes (a voxel-major copy of G,
 * Q(Q+1)/2 * N * 8 bytes), 256-byte aligned; the call allocates nothing. */
pisco_status_t pisco_eig_sets_workspace_size(int32_t Q, int64_t N, size_t* bytes);
pisco_status_t pisco_eig_sets(pisco_handle_t handle, int32_t Q, int64_t N, float bound,
                              int32_t sets, int32_t krylov, const void* G, void* maps,
                              float* lam, float* resid, void* workspace,
                              size_t workspace_bytes);

/* Many small partial SVDs at once (locally low-rank models, which Sec. I
 * and Sec. V name as beneficiaries of the method's batched small
 * eigen-problems).  For B Casorati matrices X_b of m rows and Q columns the
 * `rank` largest singular values and right singular vectors come from the
 * r largest eigenpairs of the Gram X_b^H X_b (FP32) by the per-voxel
 * Lanczos solver with a full basis; sigma_k is resolved to about
 * eps sigma_1^2 / sigma_k.
 *   X     : float2 [B][Q][m] (column q of patch b contiguous)
 *   sigma : float [rank][B], descending
 *   V     : float2 [rank][Q][B], right singular vectors (may be NULL)
 *   Xr    : float2 [B][Q][m], the rank-`rank` part X_b V V^H (may be NULL)
 *   rank  : 1..min(8, Q);  Q : 2..32
 * Workspace: pisco_llr_workspace_size. */
pisco_status_t pisco_llr_workspace_size(int64_t B, int32_t Q, int32_t rank, size_t* bytes);
pisco_status_t pisco_llr_svd(pisco_handle_t handle, int64_t B, int32_t m, int32_t Q,
                             int32_t rank, const void* X, float* sigma, void* V, void* Xr,
                             void* workspace, size_t workspace_bytes);

/* Image-support mask (Sec. III-D, the optional last step of the naive
 * algorithm).  Inside the support H(x) has rank Q - 1 and lambda_min(G(x))
 * (its smallest singular value squared) is about zero; outside it is
 * clearly positive (Sec. III-B, III-C).  The low-resolution map
 * lambda_min / |Lambda| is brought to grid_out by the periodic sinc
 * interpolation of pisco_maps, in FP64, and a voxel is inside where the
 * interpolated value is below `thresh` (in (0, 1)).
 *   lam_min : float [N_lr], e.g. from pisco_eig or pisco_estimate
 *   mask    : uint8 [grid_out], 1 inside, 0 outside
 * Workspace: pisco_workspace_size(..., PISCO_STAGE_MASK, ...). */
pisco_status_t pisco_support_mask(pisco_handle_t handle, const pisco_problem_t* prob,
                                  const float* lam_min, float thresh, uint8_t* mask,
                                  void* workspace, size_t workspace_bytes);

/* ESPIRiT's operator B(x) = I - G(x) / bound (Eq. 20; bound = |Lambda|):
 * its eigenvector for the eigenvalue one (its largest) is the map.
 *   G, B : float2 packed as from pisco_gx, N voxels (B may alias G). */
pisco_status_t pisco_espirit_operator(pisco_handle_t handle, int32_t Q, int64_t N,
                                      float bound, const void* G, void* B);

/* ---- Batches in one graph launch (not in the paper) ---------------------
 * Many problems (slices or scans of any sizes and channel counts) run as
 * one captured HIP graph, launched with a single call.  pisco_batch_create
 *  1. times candidate nullspace block sizes (the automatic one and +32,
 *     widened by 32 up to +96 while none converges) and product-kernel wave
 *     counts (1024, 2048, 4096) per distinct problem shape (eager runs on
 *     the first slice of that shape; results cached in the handle) and
 *     keeps the fastest that converges,
 *  2. runs each slice once eagerly to fix its number of nullspace products
 *     (a slice whose signal rank reaches the tuned block is given a block
 *     wider by 32 until it fits or the limit is reached),
 *  3. captures every slice's whole path with that fixed schedule (no host
 *     read-back) on up to 4 internal streams forked from one origin stream.
 * A graph launch recomputes all maps from the ACS buffers' current
 * contents; a slice whose data need more products than planned is flagged
 * PISCO_FLAG_NOT_CONVERGED in the handle's status.  The buffers passed at
 * creation (ACS, outputs, workspace) must stay allocated until
 * pisco_batch_destroy.  The eager runs of creation already write the outputs. */
typedef struct pisco_batch_s* pisco_batch_t;

/* Workspace bytes for a batch (host-only); opts may be NULL (defaults) or
 * an array of B options. */
pisco_status_t pisco_batch_workspace_size(int32_t B, const pisco_problem_t* probs,
                                          const pisco_opts_t* opts, size_t* bytes);

/*   acs[i]      : device float2 [Q][acs] of slice i
 *   maps_out[i] : device float2 [Q][grid_out] of slice i
 *   lam_min     : NULL, or an array of B device float [N_lr] (entries may be NULL)
 *   workspace   : 256-byte aligned, pisco_batch_workspace_size bytes */
pisco_status_t pisco_batch_create(pisco_handle_t handle, int32_t B,
                                  const pisco_problem_t* probs,
                                  const pisco_opts_t* opts, const void* const* acs,
                                  void* const* maps_out, float* const* lam_min,
                                  void* workspace, size_t workspace_bytes,
                                  pisco_batch_t* batch);

/* One launch of the whole batch on the handle's stream. */
pisco_status_t pisco_batch_launch(pisco_batch_t batch);

/* The tuned block size, planned product count and product wave target of
 * slice i (host-only). */
pisco_status_t pisco_batch_slice_info(pisco_batch_t batch, int32_t i, int32_t* block,
                                      int32_t* products, int32_t* ax_waves);

pisco_status_t pisco_batch_destroy(pisco_batch_t batch);

/* ---- Learned warm start (not in the paper) ------------------------------
 * A network predicts each voxel's start vector for the power iteration from
 * G(x) / |Lambda| (upper triangle: Q real diagonal entries, then Re and Im of
 * the entries p < q in row-major order) and a neighbour vector n (Re, Im):
 * two ReLU layers of 256, output y (2Q reals), start vector n + y.
 * Parameters, one flat vector (FP32 master and FP16 copy, same layout):
 *   [W1 (256 x Din, row-major), b1 (256), W2 (256 x 256), b2 (256),
 *    W3 (2Q x 256), b3 (2Q)],  Din = Q^2 + 2Q.
 * Products run on FP16 matrix cores with FP32 accumulation.  All pointers
 * are device pointers owned by the caller; Q in [2, 32]. */

/* Number of parameters (host-only). */
pisco_status_t pisco_ws_param_count(int32_t Q, int64_t* count);

/* Workspace bytes for pisco_ws_forward / pisco_ws_train_step on N voxels
 * (host-only). */
pisco_status_t pisco_ws_workspace_size(int32_t Q, int64_t N, size_t* bytes);

/* Deterministic He-uniform initialisation from `seed` (output layer scaled
 * by 1e-2, biases zero) of master (float [count]) and weights16 (FP16
 * [count]). */
pisco_status_t pisco_ws_init(pisco_handle_t handle, int32_t Q, uint64_t seed,
                             float* master, void* weights16);

/* Neighbour vectors for the grid grid_lr (z, y, x) from eigenvectors on the
 * grid coarser by two, ceil(grid_lr / 2) per dimension: voxel i takes the
 * coarse voxel floor((i - floor(lr/2)) / 2) + floor(lc/2) (the nearest
 * sample at or below its position), with the largest-magnitude entry
 * rotated to be real and positive.
 *   coarse   : float2 [Q][Nc];  neighbor : float2 [Q][N] */
pisco_status_t pisco_ws_neighbor(pisco_handle_t handle, int32_t Q,
                                 const int32_t grid_lr[3], const void* coarse,
                                 void* neighbor);

/* Start vectors init = normalise(n + y) for N voxels.
 *   G : packed as from pisco_gx;  neighbor, init : float2 [Q][N];
 *   weights16 : FP16 parameters. */
pisco_status_t pisco_ws_forward(pisco_handle_t handle, int32_t Q, int64_t N,
                                float bound, const void* G, const void* neighbor,
                                const void* weights16, void* init,
                                void* workspace, size_t workspace_bytes);

/* One training step on a batch of N >= 1 voxels with target eigenvectors
 * (float2 [Q][N], unit norm): loss 1 - |c_hat^H c|^2 / ||c_hat||^2 averaged
 * over the batch, its gradient, and, when step >= 1, one Adam update
 * (beta 0.9 / 0.999, eps 1e-8, bias correction for step `step`) of master,
 * adam_m, adam_v (float [count]) with the FP16 copy refreshed.
 *   loss_out : device float[1], the mean loss before the update (nullable)
 *   grad_out : device float[count], gradient of the SUMMED loss (nullable) */
pisco_status_t pisco_ws_train_step(pisco_handle_t handle, int32_t Q, int64_t N,
                                   float bound, const void* G,
                                   const void* neighbor, const void* target,
                                   float* master, void* weights16,
                                   float* adam_m, float* adam_v, int32_t step,
                                   float lr, float* loss_out, float* grad_out,
                                   void* workspace, size_t workspace_bytes);

/* The whole path: pisco_gram, pisco_nullspace, pisco_gx, pisco_eig and
 * pisco_maps chained, intermediates in the workspace.
 *   lam_min : float [N_lr] (may be NULL) */
pisco_status_t pisco_estimate(pisco_handle_t handle,
                              const pisco_problem_t* prob,
                              const pisco_opts_t* opts, const void* acs,
                              void* maps_out, float* lam_min, void* workspace,
                              size_t workspace_bytes);

/* Kernel tracing (measurement aid).  While enabled, every kernel launch whose
 * name contains `filter` (every launch when filter is NULL or empty) is
 * bracketed by HIP events recorded on the handle's stream.  Adds two event
 * records per traced launch; off by default. */
pisco_status_t pisco_trace_enable(pisco_handle_t handle, int32_t enable,
                                  const char* filter);

typedef struct {
  char name[64];      /* kernel name as written in the source */
  int32_t launches;   /* traced launches since the last read */
  double total_ms;    /* summed event-to-event durations */
} pisco_trace_entry_t;

/* Synchronises the handle's stream, aggregates the traced launches by kernel
 * name into `out` (host array of `cap` entries, sorted by name), writes the
 * number of distinct kernels to *count (which may exceed cap) and clears the
 * records. */
pisco_status_t pisco_trace_read(pisco_handle_t handle, pisco_trace_entry_t* out,
                                int32_t cap, int32_t* count);

#ifdef __cplusplus
}
#endif

#endif /* PISCO_H */
