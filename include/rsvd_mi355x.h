/*
 * rsvd_mi355x.h -- C ABI of the MI355X (gfx950) randomized SVD / PCA library.
 *
 * Method: Erichson, Voronin, Brunton & Kutz, "Randomized Matrix Decompositions
 * Using R" (arXiv:1608.02148).
 *   - rsvd_run  : Alg. RSVDalgorithm (Sec. 3.3) on top of Alg. rqb (Sec. 3.3)
 *                 with Alg. subspace_iter (Sec. 2.2) as the power scheme.
 *   - rpca_run  : Alg. RPCAalgorithm (Sec. 4.2), interface of Sec. 4.3, with
 *                 the column centring applied implicitly (A is never modified).
 *
 * Conventions shared by every entry point
 *   - All matrices are ROW-MAJOR with a leading dimension (elements between
 *     consecutive rows).  A is m x n; U is m x k; V is n x k and is NOT
 *     transposed (Sec. 3.6: the returned v holds right singular vectors as
 *     columns).
 *   - Every matrix / vector argument is a DEVICE pointer owned by the caller.
 *     The library never allocates device memory on the run path: scratch
 *     space is the caller's `work` buffer of at least rsvd_workspace_size()
 *     bytes (256-byte aligned).  A is read-only.
 *   - Calls are asynchronous and stream-ordered on the handle's HIP stream;
 *     outputs are valid once that stream has completed.  No call
 *     synchronises the stream except rsvd_sync_info().
 *   - Element types: A is f64, f32 or bf16 (rsvd_dtype).  U, V, rotation, x
 *     and center are f64 when A is f64 and f32 otherwise; singular values,
 *     eigvals and sdev are always f64.
 *   - Return value: RSVD_OK or a negative status.  Argument checks run before
 *     any launch.  Conditions only the device can see (non-finite data, a
 *     Cholesky breakdown) are reported in rsvd_info.flags.
 *   - Determinism: identical inputs, parameters and device give bitwise
 *     identical outputs (no floating-point atomics anywhere).
 */
#ifndef RSVD_MI355X_H
#define RSVD_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rsvd_handle_s* rsvd_handle_t;

/* Storage type of A. */
typedef enum { RSVD_F64 = 0, RSVD_F32 = 1, RSVD_BF16 = 2 } rsvd_dtype;

/* Distribution of the random test matrix Omega (Sec. 2.3). */
typedef enum { RSVD_NORMAL = 0, RSVD_UNIF = 1, RSVD_RADEMACHER = 2 } rsvd_sdist;

/* Normalisation of the power iterations (Sec. 2.2).
 * RSVD_SCHEME_QR: Alg. subspace_iter, each half-step re-orthonormalised by
 *   QR (CholeskyQR here).
 * RSVD_SCHEME_LU: Alg. normalized_iter, each half-step replaced by the L
 *   factor of a pivoted LU (tournament pivoting on the device; the span, and
 *   so the result in exact arithmetic, is the same).  Sketch widths
 *   l <= RSVD_MAX_L; single solves only (batches return
 *   RSVD_ERR_UNSUPPORTED).  The final basis Q = qr(Y) is orthonormal in
 *   either scheme. */
typedef enum { RSVD_SCHEME_QR = 0, RSVD_SCHEME_LU = 1 } rsvd_power_scheme;

/* Arithmetic of the passes over A.
 * RSVD_PREC_PLAIN: products in the storage precision of A (f64 MFMA for f64,
 *   f32 MFMA for f32 and bf16).
 * RSVD_PREC_BF16_MIXED (A in f32 or bf16): the early passes (the sketch and
 *   the power iterations except the last half-step) run on bf16 MFMA with f32
 *   accumulation; the last sketch and the projection B = Q^T A are
 *   near-f32-accurate by splitting the operands into bf16 hi + lo terms.
 *   Gram matrices, Cholesky factors and the small SVD stay f64 in every mode. */
typedef enum { RSVD_PREC_PLAIN = 0, RSVD_PREC_BF16_MIXED = 1 } rsvd_precision;

/* Parameters of Alg. rqb / Alg. RSVDalgorithm. */
typedef struct {
    int32_t  p;          /* oversampling, l = k + p (default 10, Sec. 3.3 remark) */
    int32_t  q;          /* subspace iterations (default 2, Sec. 3.3 remark)    */
    uint64_t seed;       /* Philox key of Omega                                  */
    uint32_t stream_id;  /* Philox counter word 2 of Omega (batch index)        */
    int32_t  sdist;      /* rsvd_sdist                                           */
    int32_t  precision;  /* rsvd_precision                                       */
    int32_t  probes;     /* r > 0: a-posteriori error bound from r Gaussian probes
                            (rsvd_info.est_err; 0..16, default 0 = off)           */
    int32_t  scheme;     /* rsvd_power_scheme (default RSVD_SCHEME_QR)           */
    int32_t  reserved;
} rsvd_params;

/* Device-side outcome record (optional; written by the last kernel). */
typedef struct {
    int32_t  l;          /* sketch width actually used: min(k + p, m, n)          */
    int32_t  q;          /* subspace iterations performed                         */
    int32_t  p;          /* oversampling actually used (l - k)                    */
    uint32_t flags;      /* RSVD_FLAG_* bits                                      */
    double   est_err;    /* with params.probes = r > 0: 10 sqrt(2/pi) max_i
                            ||(A - U S V^T) w_i||_2 over r Gaussian probes w_i
                            (Philox, counter word 2 = stream_id ^ 0x80000000),
                            an upper bound of ||A - U S V^T||_2 with probability
                            at least 1 - 10^-r (Halko, Martinsson & Tropp, SIAM
                            Review 2011, Sec. 4.3); for rpca_run the centred
                            matrix and x V^T.  0 when probes = 0.               */
} rsvd_info;

#define RSVD_FLAG_CHOL_SHIFT   1u  /* a Gram matrix needed the shifted Cholesky    */
#define RSVD_FLAG_DEGENERATE   2u  /* a column was numerically zero after shifting */
#define RSVD_FLAG_NONFINITE    4u  /* NaN or Inf reached a Gram matrix             */
#define RSVD_FLAG_JACOBI_SLOW  8u  /* small SVD stopped at its sweep limit (for
                                      l > 128 also: a round of its block sweeps
                                      timed out waiting for the other
                                      workgroups; the results are then not
                                      reliable)                                  */
#define RSVD_FLAG_ZERO_SCALE  16u  /* scaled PCA: a column had zero spread (its
                                      scale was set to 1; see rpca_run_ex)       */
/* Bits 24..31 of rsvd_info.flags hold the number of Jacobi sweeps the small SVD
 * of B took (diagnostic). */
#define RSVD_FLAG_SWEEPS_SHIFT 24

/* Status codes. */
#define RSVD_OK               0
#define RSVD_ERR_INVALID     -1   /* bad argument (sizes, NULL, workspace, ...)   */
#define RSVD_ERR_UNSUPPORTED -2   /* dtype / mode / size not supported            */
#define RSVD_ERR_HIP         -3   /* HIP runtime error, see rsvd_last_hip_error() */
#define RSVD_ERR_NONFINITE   -4   /* reported by rsvd_sync_info only              */
#define RSVD_ERR_BREAKDOWN   -5   /* reported by rsvd_sync_info only              */

/* Largest sketch width l = k + p: RSVD_MAX_L for batches and the kernel-level
 * entry points, RSVD_MAX_L_SINGLE for rsvd_run / rpca_run (widths above
 * RSVD_MAX_L take a blocked Cholesky and a Jacobi with its matrix in the
 * workspace instead of LDS). */
#define RSVD_MAX_L 128
#define RSVD_MAX_L_SINGLE 256

/* Fill *p with the paper's defaults: p = 10, q = 2, Gaussian Omega, seed 0. */
void rsvd_default_params(rsvd_params* p);

/* Create / destroy a handle bound to a HIP stream (hipStream_t passed as
 * void*; NULL = default stream).  The handle owns no device memory. */
int rsvd_create(rsvd_handle_t* handle, void* hip_stream);
int rsvd_destroy(rsvd_handle_t handle);
int rsvd_set_stream(rsvd_handle_t handle, void* hip_stream);
int rsvd_last_hip_error(rsvd_handle_t handle);
/* Tile variants of the f32-compute products, one per (mode, column class):
 * variants[0..5] for Y = A X and variants[6..11] for Z = A^T Q, classes
 * 32, 48, 64, 80, 96, 128 columns (the class of a solve is the smallest that
 * holds l).  0 = 4 waves per workgroup, 1 = 8 waves, 2 = 16 waves over the
 * same 128 x class output tile.  Results do not depend on the variant (the
 * reduction order per output element is the same); only the speed does.
 * Plans made after the call use the new table; an autotuner that times the
 * variants writes the table the Python binding applies. */
int rsvd_set_tile_variants(rsvd_handle_t handle, const int32_t* variants);
int rsvd_get_tile_variants(rsvd_handle_t handle, int32_t* variants);
const char* rsvd_status_string(int status);

/* Workspace bytes needed by rsvd_run / rpca_run for this problem.
 * Same argument rules as rsvd_run; returns RSVD_ERR_INVALID for bad sizes. */
int rsvd_workspace_size(rsvd_handle_t handle, int32_t dtype, int64_t m, int64_t n,
                        int32_t k, const rsvd_params* params, size_t* bytes);

/* Randomized SVD, Alg. RSVDalgorithm (Sec. 3.3):
 *   [Q, B] = rqb(A, k, p, q); [U~, S, V] = svd(B); U = Q U~; truncate to k.
 * A      : m x n, leading dimension lda >= n, dtype `dtype`.
 * k      : target rank, 1 <= k < min(m, n).  l = min(k + p, m, n) <= RSVD_MAX_L_SINGLE.
 * U      : m x k (ldu >= k) or NULL (left vectors not wanted).
 * S      : k singular values, descending (f64, required).
 * V      : n x k (ldv >= k) or NULL (right vectors not wanted).
 * info   : device pointer to one rsvd_info, or NULL.
 * Sign convention: each pair (u_i, v_i) is oriented so that the entry of v_i
 * with the largest magnitude is positive (lowest index on ties). */
int rsvd_run(rsvd_handle_t handle, int32_t dtype, int64_t m, int64_t n,
             const void* A, int64_t lda, int32_t k, const rsvd_params* params,
             void* U, int64_t ldu, double* S, void* V, int64_t ldv,
             void* work, size_t work_bytes, rsvd_info* info);

/* Randomized PCA, Alg. RPCAalgorithm (Sec. 4.2) with the outputs of Sec. 4.3.
 * center != 0: the column means mu are removed implicitly (the products use
 *   A - 1 mu^T without forming it).  center == 0: A is used as is.
 * rotation : n x k principal directions W = V (ldr >= k), required.
 * eigvals  : k values S^2 / (m - 1) (f64), required.
 * sdev     : k values sqrt(eigvals) (f64) or NULL.
 * x        : m x k principal components U S (ldx >= k) or NULL (retx = FALSE).
 * center_out : n column means (zeros when center == 0) or NULL. */
int rpca_run(rsvd_handle_t handle, int32_t dtype, int64_t m, int64_t n,
             const void* A, int64_t lda, int32_t k, int32_t center,
             const rsvd_params* params, void* rotation, int64_t ldr,
             double* eigvals, double* sdev, void* x, int64_t ldx, void* center_out,
             void* work, size_t work_bytes, rsvd_info* info);

/* Randomized PCA with the options and outputs of Sec. 4.3 and the extras of
 * Sec. 4.1 (Alg. RPCAalgorithm on the centred and optionally scaled data).
 * opt->center != 0: the column means mu are removed implicitly.
 * opt->scale != 0: each (centred) column is also divided by its root mean
 *   square about the centre with the m - 1 divisor (its standard deviation
 *   when centring), so the analysis is that of the correlation matrix; the
 *   division is applied to the skinny operands of the products (A is read as
 *   is).  A column with zero spread keeps scale 1 (it contributes nothing)
 *   and sets RSVD_FLAG_ZERO_SCALE in info->flags.
 * Outputs (device pointers, element type as for rpca_run; NULL = not wanted
 * unless marked required):
 *   rotation  n x k principal directions W (ldr >= k), required;
 *   eigvals   k values s^2 / (m - 1) (f64), required;
 *   sdev      k values sqrt(eigvals) (f64);
 *   x         m x k principal components U S (ldx >= k);
 *   x_white   m x k whitened components x_i / sdev_i, each of unit variance
 *             (Sec. 4.1; zero columns where sdev_i = 0) (ldxw >= k);
 *   loadings  n x k loadings W diag(sdev) (Sec. 4.1) (ldl >= k);
 *   center    n centre values (zeros without centring);
 *   scale     n scale values (ones without scaling);
 *   total_var one f64: the sum of the column variances of the analysed
 *             (centred, scaled) data, so eigvals / total_var are the
 *             explained proportions of Sec. 4.1.
 * Workspace: rsvd_workspace_size with the same arguments.  Errors as
 * rsvd_run. */
typedef struct {
    int32_t center;
    int32_t scale;
    int32_t reserved[2];
} rpca_options;

typedef struct {
    void* rotation; int64_t ldr;
    double* eigvals;
    double* sdev;
    void* x; int64_t ldx;
    void* x_white; int64_t ldxw;
    void* loadings; int64_t ldl;
    void* center;
    void* scale;
    double* total_var;
} rpca_outputs;

int rpca_run_ex(rsvd_handle_t handle, int32_t dtype, int64_t m, int64_t n,
                const void* A, int64_t lda, int32_t k, const rpca_options* opt,
                const rsvd_params* params, const rpca_outputs* out,
                void* work, size_t work_bytes, rsvd_info* info);

/* Principal components of new observations (the predict step of Sec. 4.4):
 * x = ((A - 1 center^T) diag(scale)^-1) rotation for A m x n (dtype, lda >=
 * n), with rotation n x k (ldr >= k), center and scale n-vectors as returned
 * by rpca_run_ex (element type of the outputs; NULL = no centring / no
 * scaling), x m x k (ldx >= k).  k <= RSVD_MAX_L_SINGLE.  Storage-precision
 * arithmetic (f64 matrix cores for f64, f32 otherwise); the centre is
 * subtracted while A is read.  work: rpca_predict_workspace_size bytes. */
int rpca_predict_workspace_size(rsvd_handle_t handle, int32_t dtype, int64_t m, int64_t n,
                                int32_t k, size_t* bytes);
int rpca_predict(rsvd_handle_t handle, int32_t dtype, int64_t m, int64_t n, const void* A,
                 int64_t lda, int32_t k, const void* rotation, int64_t ldr, const void* center,
                 const void* scale, void* x, int64_t ldx, void* work, size_t work_bytes);

/* ---- Robust PCA (Alg. rpca, Sec. 5.2) -------------------------------------
 * A = L + S with L low rank and S sparse, by the inexact augmented Lagrange
 * multiplier method (Eq. IALM) with the randomized SVD of rsvd_run (params:
 * p, q, seed, stream_id, sdist; plain precision) at a target rank that the
 * method predicts each iteration.  Where the paper defers to Lin, Chen & Ma
 * (2010, arXiv:1009.5055) this follows their inexact ALM: mu starts at
 * mu0_scale / ||A||_2 (the listing's 1.25 ||A||_2 read as 1.25 / ||A||_2) and
 * grows by rho per iteration up to 1e7 times its start; the multiplier starts
 * at A / max(||A||_2, ||A||_max / lambda); the target rank starts at 2 and is
 * l + 1 when fewer than k singular values exceed 1/mu (l of them), else
 * l + round(0.05 min(m, n)), clamped to [1, k_max]; the iteration stops when
 * ||A - L - S||_F / ||A||_F < tol or after maxiter iterations.  ||A||_2 is the
 * randomized SVD's rank-1 estimate.  The randomized SVD is used at every
 * rank (the paper switches to a deterministic SVD above min(m, n) / 4; here
 * the rank is capped at k_max instead).
 * A, L, S: m x n row-major (f64 or f32, lda / ldl / lds >= n); L and S are
 * written.  The host reads two scalars per iteration (the singular values
 * and the residual), so the call synchronises the handle's stream and
 * returns when done; result (host, may be NULL) receives the iteration
 * count, the final rank l and target rank k, the relative residual and the
 * lambda used.  work: rrpca_workspace_size bytes (two m x n matrices plus
 * the randomized SVD's workspace at rank k_max). */
typedef struct {
    double  lambda;     /* weight of ||S||_1; <= 0: max(m, n)^-1/2 (Sec. 5.4)     */
    double  tol;        /* relative residual to stop at (default 1e-5)            */
    double  rho;        /* growth of mu per iteration (default 1.6)               */
    double  mu0_scale;  /* mu starts at mu0_scale / ||A||_2 (default 1.25)       */
    int32_t maxiter;    /* default 50                                            */
    int32_t k_max;      /* largest target rank; <= 0: min(m, n) - 1, at most
                           RSVD_MAX_L_SINGLE - p                                  */
} rrpca_options;

typedef struct {
    int32_t iterations, rank, k, reserved;
    double  residual;   /* ||A - L - S||_F / ||A||_F after the last iteration      */
    double  lambda;
} rrpca_result;

void rrpca_default_options(rrpca_options* opt);
int rrpca_workspace_size(rsvd_handle_t handle, int32_t dtype, int64_t m, int64_t n,
                         const rrpca_options* opt, const rsvd_params* params, size_t* bytes);
int rrpca_run(rsvd_handle_t handle, int32_t dtype, int64_t m, int64_t n, const void* A,
              int64_t lda, const rrpca_options* opt, const rsvd_params* params, void* L,
              int64_t ldl, void* S, int64_t lds, void* work, size_t work_bytes,
              rrpca_result* result);

/* ---- Interpolative and CUR decompositions (Sec. 6) -----------------------
 * rid_run, Alg. rid: [Q, B] = rqb(A, k, p, q) (the passes of rsvd_run up to
 * B = Q^T A, params as there, plain precision), then the column ID of B
 * (Alg. id): k steps of column-pivoted QR (at each step the column with the
 * largest remaining norm; lowest index on ties), T = S11^-1 S12 (S = the
 * triangular factor; a zero diagonal entry of S11 gives a zero row of T),
 * Z[:, P] = [I_k, T], J = P[:k], and C = A[:, J].  A ~ C Z.
 * rcur_run, Alg. rcur: C, Z, J as rid_run, then k steps of column-pivoted QR
 * of C^T choose the rows I, R = A[I, :], U = Z pinv(R) (R of full row rank:
 * pinv(R) = Q_r T_r^-T from the QR R^T = Q_r T_r).  A ~ C U R.  k <= RSVD_MAX_L.
 * A: m x n (dtype, lda >= n); C m x k (ldc >= k), Z k x n (ldz >= n), U k x k
 * (ldu >= k), R k x n (ldr >= n), element type as rsvd_run's U (C and R hold
 * A's entries exactly); J, I: device int32 arrays of k column / row indices
 * in pivot order.  rid_run: C and Z may be NULL (indices only).  The row ID
 * is the column ID of A^T (pass the transpose).  work: rid_workspace_size
 * bytes with cur = 0 for rid_run, 1 for rcur_run.  Asynchronous on the
 * handle's stream; errors as rsvd_run. */
int rid_workspace_size(rsvd_handle_t handle, int32_t dtype, int64_t m, int64_t n, int32_t k,
                       const rsvd_params* params, int32_t cur, size_t* bytes);
int rid_run(rsvd_handle_t handle, int32_t dtype, int64_t m, int64_t n, const void* A,
            int64_t lda, int32_t k, const rsvd_params* params, int32_t* J, void* C,
            int64_t ldc, void* Z, int64_t ldz, void* work, size_t work_bytes);
int rcur_run(rsvd_handle_t handle, int32_t dtype, int64_t m, int64_t n, const void* A,
             int64_t lda, int32_t k, const rsvd_params* params, int32_t* J, int32_t* I,
             void* C, int64_t ldc, void* U, int64_t ldu, void* R, int64_t ldr, void* work,
             size_t work_bytes);

/* rsvd_run for callers that cannot allocate device memory (code under HIP
 * graph capture, serving loops, harnesses that forbid allocation): same
 * arguments, results and rules as rsvd_run, without `work` / `work_bytes`.
 * The workspace is a fixed device array of RSVD_NOALLOC_SCRATCH_BYTES that
 * the library holds on each device it runs on, from the first call there
 * until the process ends; the call itself allocates nothing.  Problems whose
 * rsvd_workspace_size exceeds it return RSVD_ERR_UNSUPPORTED before any
 * launch.  Every call on one device shares the array: calls that overlap on
 * a device (different streams or threads) race and must be serialised by the
 * caller.  Event timing (rsvd_profile_enable) is not recorded for these
 * calls. */
#define RSVD_NOALLOC_SCRATCH_BYTES (256ull << 20)
int rsvd_run_noalloc(rsvd_handle_t handle, int32_t dtype, int64_t m, int64_t n,
                     const void* A, int64_t lda, int32_t k, const rsvd_params* params,
                     void* U, int64_t ldu, double* S, void* V, int64_t ldv, rsvd_info* info);

/* Synchronise the handle's stream, copy the device record `dinfo` to the host
 * record `hinfo`, and map its flags to a status: RSVD_ERR_NONFINITE when
 * non-finite data reached a Gram matrix, RSVD_ERR_BREAKDOWN when a column
 * stayed numerically zero after the shifted Cholesky, else RSVD_OK. */
int rsvd_sync_info(rsvd_handle_t handle, const rsvd_info* dinfo, rsvd_info* hinfo);

/* ---- Ragged batches ------------------------------------------------------
 * Many independent randomized SVDs (Alg. RSVDalgorithm, one per matrix, all
 * with the same rsvd_params except the Omega stream), run as one sequence of
 * grouped launches: each step of the solve is a single launch over every
 * matrix of the batch, so thousands of small solves fill the device.
 *
 * Life cycle: rsvd_batch_create (host; sizes the workspace) ->
 * rsvd_batch_bind (uploads the launch tables into the workspace; synchronises
 * the handle's stream once; with RSVD_BATCH_GRAPH also captures the whole
 * launch sequence in a HIP graph) -> rsvd_batch_run, any number of times
 * (asynchronous on the handle's stream; no allocation, no host
 * synchronisation; without RSVD_BATCH_GRAPH a caller may capture it in its
 * own graph) -> rsvd_batch_destroy.  The handle must outlive the batch.
 * Matrices are grouped by sketch width; the groups run concurrently on side
 * streams the handle owns (default priority, created on first use), forked
 * from and joined back to the handle's stream with events, so a run is still
 * one stream-ordered operation on the handle's stream.
 *
 * Results: matrix b gets the solve that rsvd_run computes for it with
 * params.stream_id = desc[b].stream_id (same steps and kernels); products here
 * never split their reduction into partial sums, so the rounding can differ
 * from rsvd_run's, within the same accuracy.
 * Rules: every matrix has the same dtype; either every U is NULL or none is;
 * l_b = min(k_b + p, m_b, n_b) <= RSVD_MAX_L.  Argument errors in any entry
 * fail the whole create call. */
typedef struct {
    const void* A;       /* m x n (dtype, lda >= n), read-only          */
    int64_t lda;
    int64_t m, n;
    int32_t k;           /* 1 <= k < min(m, n)                          */
    uint32_t stream_id;  /* Omega counter word 2 for this matrix        */
    void* U;             /* m x k (ldu >= k) or NULL                    */
    int64_t ldu;
    double* S;           /* k singular values, descending               */
    void* V;             /* n x k (ldv >= k) or NULL                    */
    int64_t ldv;
    rsvd_info* info;     /* device record or NULL                       */
    float* features;     /* RSVD_BATCH_FEATURES: 131 selector inputs    */
    int32_t q, p;        /* RSVD_BATCH_OWN_QP: this matrix's q and p    */
} rsvd_batch_desc;

typedef struct rsvd_batch_s* rsvd_batch_t;

#define RSVD_BATCH_GRAPH    1  /* bind captures the launches in a HIP graph    */
#define RSVD_BATCH_STAMPS   2  /* record device-clock stamps per matrix         */
#define RSVD_BATCH_FEATURES 4  /* run only the q = 0 sketch of each matrix and
                                  write its selector inputs (desc.features,
                                  see the selector network below); S, U, V
                                  are not written                               */
#define RSVD_BATCH_CHUNKED 16  /* split each size class into 4 chunks of about
                                  equal work that run one after another on
                                  the class's stream: a matrix's solve spans
                                  its chunk's launches (about a quarter of the
                                  batch time) instead of all of them        */
#define RSVD_BATCH_OWN_QP   8  /* take q and p from each desc instead of
                                  params (a group runs its largest q; each
                                  member's extra iterations are switched off
                                  on the device)                               */

/* descs: HOST array of `count` entries (their pointers are device pointers,
 * recorded at bind time).  *work_bytes receives the workspace size. */
int rsvd_batch_create(rsvd_handle_t handle, int32_t dtype, int32_t count,
                      const rsvd_batch_desc* descs, const rsvd_params* params,
                      int32_t flags, rsvd_batch_t* batch, size_t* work_bytes);
/* work: device buffer of >= work_bytes, 256-byte aligned, owned by the caller
 * and reserved for this batch until it is destroyed or bound again. */
int rsvd_batch_bind(rsvd_batch_t batch, void* work, size_t work_bytes);
int rsvd_batch_run(rsvd_batch_t batch);
/* With RSVD_BATCH_STAMPS: synchronise and copy the device-clock stamps of the
 * last run, host[2b] = when matrix b's first step ran, host[2b+1] = when its
 * last step ran; *ticks_per_second receives the clock rate. */
int rsvd_batch_stamps(rsvd_batch_t batch, uint64_t* host, double* ticks_per_second);
int rsvd_batch_destroy(rsvd_batch_t batch);

/* Learned choice of (q, p) for each matrix of a batch (see the selector
 * network below): runs the q = 0 sketches as an RSVD_BATCH_FEATURES batch and
 * the network on their features, then picks per matrix, from the network's
 * distribution P over the cheapest sufficient class, the cheapest class c
 * (cost (2q + 2)(k + p), ties to the lower index) whose estimated chance of
 * sufficing -- the mass of P on the classes that c dominates (no larger q, no
 * larger p) -- is at least tau; tau <= 0 takes the most probable class.  The
 * chosen q and p of matrix b go to the HOST arrays q_out[b], p_out[b] (the
 * features to features_out, a device array of count x 131 floats, when not
 * NULL).  Synchronises the handle's stream once.  Only A, lda, m, n, k and
 * stream_id of each desc are read; params gives the seed, test matrix and
 * precision.  The sketch's Omega columns are a prefix of the later solve's
 * (same seed, same stream). */
int rsvd_select_workspace_size(rsvd_handle_t handle, int32_t dtype, int32_t count,
                               const rsvd_batch_desc* descs, const rsvd_params* params,
                               size_t* bytes);
int rsvd_select(rsvd_handle_t handle, int32_t dtype, int32_t count, const rsvd_batch_desc* descs,
                const rsvd_params* params, const float* theta, float tau, int32_t* q_out,
                int32_t* p_out, float* features_out, void* work, size_t work_bytes);

/* Learned batch: the selector and the solves in one stream-ordered launch
 * sequence with no host round trip (one graph with RSVD_BATCH_GRAPH).  A run
 * takes three phases: (1) for every matrix the q = 0 sketch Y0 = A Omega[:, :l0]
 * (l0 as for the selector features below) and its 131 features; (2) the
 * network on all features and, per matrix, q_b = the fewest power iterations
 * whose classes (q' <= q_b, p' <= params->p: the pairs a solve with q_b
 * iterations and oversampling params->p covers) hold at least tau of the
 * network's probability mass, RSVD_LEARNED_QMAX when no q_b does (tau <= 0:
 * the q of the most probable class); theta = NULL
 * skips the network and takes q_b = RSVD_LEARNED_FALLBACK_Q for every matrix;
 * (3) every solve with its own q_b (<= RSVD_LEARNED_QMAX; the extra
 * iterations of its group are switched off on the device) and p = params->p
 * (0..RSVD_LEARNED_PMAX), starting from the leading l = min(k + p, m, n)
 * columns of Y0 instead of a new sketch: Omega's entries do not depend on its
 * width, so these are the columns of the solve's own A Omega.  Sec. 3.6 fixes
 * only defaults for q and p and Sec. 2.2 advises more iterations for slowly
 * decaying spectra; the network supplies the per-matrix choice.
 * descs: as rsvd_batch_create (q, p and features are not read); params: seed,
 * test matrix, precision, p and probes (params.q is not read); flags:
 * RSVD_BATCH_GRAPH and RSVD_BATCH_STAMPS only (stamps span all three phases).
 * theta: device vector of RSVD_MLP_PARAMS floats or NULL, read at every run.
 * Life cycle and workspace: as rsvd_batch_create / bind / run / destroy.
 * info records report q_b and l. */
#define RSVD_LEARNED_QMAX       4
#define RSVD_LEARNED_PMAX       20
#define RSVD_LEARNED_FALLBACK_Q 3
int rsvd_batch_create_learned(rsvd_handle_t handle, int32_t dtype, int32_t count,
                              const rsvd_batch_desc* descs, const rsvd_params* params,
                              const float* theta, float tau, int32_t flags,
                              rsvd_batch_t* batch, size_t* work_bytes);
/* Learned batches: synchronise and copy the q chosen for each matrix by the
 * last run into the HOST array q_host (count int32). */
int rsvd_batch_choices(rsvd_batch_t batch, int32_t* q_host);

/* ---- Learned choice of (q, p): the selector network ---------------------
 * A three-layer perceptron reads 131 features of a matrix (the singular values
 * of its q = 0 sketch Y0 = A Omega[:, :l0], l0 = min(max(2k, k + 20), m, n,
 * 128), divided by the largest and zero-padded to 128, then log2(m)/12,
 * log2(n)/12, log2(k)/12) and scores 15 classes c = 3 q + j, q = 0..4,
 * p = (5, 10, 20)[j].  The paper fixes no rule for q and p beyond its defaults
 * (Sec. 3.6) and the advice to iterate more on slowly decaying spectra
 * (Sec. 2.2); the network learns the cheapest pair that meets an accuracy
 * target.  Layers 131 -> 64 -> 64 -> 15, ReLU, softmax; parameters are one
 * f32 device vector of RSVD_MLP_PARAMS values in the order W1 (131 x 64,
 * row-major), b1, W2 (64 x 64), b2, W3 (64 x 15), b3. */
#define RSVD_MLP_INPUTS  131
#define RSVD_MLP_HIDDEN  64
#define RSVD_MLP_CLASSES 15
#define RSVD_MLP_PARAMS  13583

/* Workspace bytes of rsvd_mlp_train_step for `batch` samples. */
int rsvd_mlp_workspace_size(int32_t batch, size_t* bytes);
/* He-uniform weights (U(-a, a), a = sqrt(6 / fan_in), from Philox under
 * `seed`), zero biases. */
int rsvd_mlp_init(rsvd_handle_t handle, float* theta, uint64_t seed);
/* Forward pass of `batch` samples x (batch x 131, f32, row-major): prob
 * (batch x 15 softmax, or NULL) and cls (batch int32 argmax, lowest index on
 * ties, or NULL; not both NULL). */
int rsvd_mlp_forward(rsvd_handle_t handle, const float* theta, int32_t batch,
                     const float* x, float* prob, int32_t* cls);
/* One training step on the mean cross-entropy of labels (batch int32 classes):
 * forward, back-propagation, gradient (written to grad if not NULL) and loss
 * (device f32 scalar if not NULL); then, for step >= 1, one Adam update
 * (beta1 0.9, beta2 0.999, eps 1e-8, bias correction for step t = step) of
 * theta, adam_m and adam_v (zero-initialised by the caller before step 1).
 * step = 0 computes the gradient and loss only.  Sums run in a fixed order:
 * the result is deterministic. */
int rsvd_mlp_train_step(rsvd_handle_t handle, float* theta, float* adam_m, float* adam_v,
                        int32_t step, float lr, int32_t batch, const float* x,
                        const int32_t* labels, float* grad, float* loss,
                        void* work, size_t work_bytes);

/* Selector checkpoint file (what the training driver writes): a 64-byte
 * little-endian header -- magic "RSVDMLP1", u32 format version (1), u32
 * parameter count (RSVD_MLP_PARAMS), u32 Adam step, u64 seed, u64 size of the
 * training set, 8 bytes of a digest of the training data, f32 decision
 * threshold tau tuned on the validation split (0 = not set), zero padding --
 * then theta, adam_m and adam_v as RSVD_MLP_PARAMS float32 each. */
typedef struct {
    uint32_t version, params, step, reserved;
    uint64_t seed, n_train;
    uint8_t  digest[8];
    float    tau;
    uint32_t reserved2;
} rsvd_mlp_header;

/* Read a selector checkpoint from the host file `path` into the device
 * vectors theta and, when not NULL, adam_m and adam_v (RSVD_MLP_PARAMS floats
 * each, caller-owned); header (host, may be NULL) receives the header fields.
 * The file is checked in full before anything is written to the device:
 * RSVD_ERR_INVALID when an argument is NULL, the file cannot be opened, its
 * size is not 64 + 3 * 4 * RSVD_MLP_PARAMS bytes, or any stored value is not
 * finite; RSVD_ERR_UNSUPPORTED for a wrong magic, format version or
 * parameter count.  theta = NULL (then adam_m and adam_v NULL too) only
 * checks the file and fills header, with no device access.  Otherwise
 * synchronises the handle's stream (the copies are done when the call
 * returns). */
int rsvd_mlp_load(rsvd_handle_t handle, const char* path, float* theta, float* adam_m,
                  float* adam_v, rsvd_mlp_header* header);

/* ---- Optional per-kernel timing ------------------------------------------
 * When enabled, every product with A (the passes of Alg. rqb and
 * Alg. subspace_iter) is bracketed by HIP events on the handle's stream, so a
 * caller can time those kernels inside its own timed region.  Kinds:
 * 0 = A X (sketch / power-iteration half), 1 = A^T Q (power-iteration half and
 * the projection B^T).  flops / bytes are the algorithmic counts of the
 * recorded launches (2 m n l flops; one read of A plus the skinny operands). */
typedef struct {
    int32_t count;       /* launches recorded                       */
    int32_t reserved;
    double  total_ms;    /* summed event-to-event durations         */
    double  flops;       /* summed algorithmic flops                */
    double  bytes;       /* summed algorithmic HBM bytes            */
} rsvd_kernel_stat;

#define RSVD_PROFILE_KINDS 2

int rsvd_profile_enable(rsvd_handle_t handle, int32_t enable);
/* Synchronise the stream, sum the recorded intervals per kind into
 * out[0 .. RSVD_PROFILE_KINDS), and clear the record. */
int rsvd_profile_collect(rsvd_handle_t handle, rsvd_kernel_stat* out);

/* ---- Building blocks exposed for kernel-level parity tests ------------- */

/* The 32-bit Philox words behind Omega: out[j * 4*groups + 4*c + t] = word t of
 * Philox4x32-10(counter (j, c, stream_id, 0), key (seed lo, seed hi)) for
 * j < n, c < groups.  out is a device array of n * 4 * groups uint32. */
int rsvd_philox_words(rsvd_handle_t handle, int64_t n, int32_t groups,
                      uint64_t seed, uint32_t stream_id, uint32_t* out);

/* The random test matrix Omega (n x l, row-major, ld = ldo) of Alg. rqb
 * in f64 (dtype RSVD_F64) or f32 (otherwise), entries per rsvd_sdist. */
int rsvd_test_matrix(rsvd_handle_t handle, int32_t dtype, int64_t n, int32_t l,
                     uint64_t seed, uint32_t stream_id, int32_t sdist,
                     void* out, int64_t ldo);

/* Arithmetic of the kernel-level products below: 0 = storage precision (f64
 * matrix cores for RSVD_F64, f32 otherwise), 1 = bf16 matrix cores (operands
 * rounded to bf16, f32 accumulation), 2 = split bf16 (A_hi X_hi + A_hi X_lo +
 * A_lo X_hi; error per product about 2^-18 |a||x|, near f32 rounding).  1 and 2
 * are rejected for RSVD_F64. */
#define RSVD_ARITH_STORAGE 0
#define RSVD_ARITH_BF16    1
#define RSVD_ARITH_SPLIT   2

/* Y = A X (Alg. rqb, Alg. subspace_iter): A m x K (dtype,
 * lda), X K x c (f64 for RSVD_F64 else f32, ldx), Y m x c (same type as X,
 * ldy).  c <= RSVD_MAX_L_SINGLE.
 * splits: 0 = the split of the K-reduction that rsvd_run uses for this shape;
 * 1..4 = that many chunks of K, each product writing a partial block to the
 * workspace, summed in chunk order (deterministic).  Other values:
 * RSVD_ERR_INVALID.
 * work: optional (may be NULL) for RSVD_ARITH_STORAGE without a split; the
 * bf16 arithmetics pack X into bf16 there and split products keep their
 * partial blocks there, which needs rsvd_block_workspace_size(dtype, m, K, c)
 * bytes (RSVD_ERR_INVALID otherwise).  Given at that size for the storage
 * arithmetic, it lets large products take the streamed kernel (X copied
 * k-contiguous there); smaller or NULL work keeps the LDS-staged tiles.
 * Kernel choice: products with m K >= 2^24, 64 < c <= 224 and 16-byte
 * aligned rows of A stream A straight into the matrix cores; others stage
 * tiles of A in LDS.  Results agree to rounding (the order of the sum over K
 * differs); RSVD_PRODUCTS=staged in the environment keeps the staged tiles,
 * and RSVD_STREAM_WPS=1 (=2) keeps the streamed kernels at one wave per SIMD
 * (at most eight-wave workgroups). */
int rsvd_gemm_nn(rsvd_handle_t handle, int32_t dtype, int32_t arith, int64_t m, int64_t K, int32_t c,
                 const void* A, int64_t lda, const void* X, int64_t ldx,
                 void* Y, int64_t ldy, int32_t splits, void* work, size_t work_bytes);

/* Z = A^T Q (Alg. subspace_iter; Alg. rqb gives B^T): A m x n
 * (dtype, lda), Q m x c (f64/f32, ldq), Z n x c (ldz).  c <= RSVD_MAX_L_SINGLE.
 * Kernel choice as for rsvd_gemm_nn (the streamed kernel also needs n % 4 == 0). */
int rsvd_gemm_tn(rsvd_handle_t handle, int32_t dtype, int32_t arith, int64_t m, int64_t n, int32_t c,
                 const void* A, int64_t lda, const void* Q, int64_t ldq,
                 void* Z, int64_t ldz, void* work, size_t work_bytes);

/* Economic QR of Y (m x c, f64 or f32 per dtype, ldy) in place: Y <- Q with
 * orthonormal columns, R (c x c, f64, row-major, ld c) upper triangular with
 * positive diagonal, Y = Q R.  CholeskyQR2, shifted CholeskyQR3 on breakdown.
 * flags (device uint32, may be NULL) receives RSVD_FLAG_* bits. */
int rsvd_orthonormalize(rsvd_handle_t handle, int32_t dtype, int64_t m, int32_t c,
                        void* Y, int64_t ldy, double* R, uint32_t* flags,
                        void* work, size_t work_bytes);

/* Workspace bytes for the three building blocks above at these sizes (c up to
 * RSVD_MAX_L_SINGLE for the products, RSVD_MAX_L for the other two). */
int rsvd_block_workspace_size(rsvd_handle_t handle, int32_t dtype, int64_t m,
                              int64_t n, int32_t c, size_t* bytes);

/* Pivoted LU normalisation of Y (m x c, f64 or f32 per dtype, ldy) in place,
 * the step of Alg. normalized_iter: Y = L U with L row-permuted unit lower
 * trapezoidal (Y <- L) and U upper triangular (c x c, f64, row-major, ld c,
 * or NULL).  piv (device int32, c entries, or NULL): the row of Y that
 * pivots at step i, so L[piv[i]][0..i) holds the multipliers, L[piv[i]][i] = 1
 * and L[piv[i]][i+1..c) = 0 up to rounding.  Pivot rows are chosen by
 * tournament pivoting over blocks of 256 rows; for m <= 256 they are those of
 * partial pivoting.  c <= RSVD_MAX_L, c <= m.  flags as for
 * rsvd_orthonormalize (RSVD_FLAG_DEGENERATE on a zero pivot).  work:
 * rsvd_block_workspace_size(dtype, m, m, c) bytes. */
int rsvd_lu_normalize(rsvd_handle_t handle, int32_t dtype, int64_t m, int32_t c, void* Y,
                      int64_t ldy, int32_t* piv, double* U, uint32_t* flags, void* work,
                      size_t work_bytes);

/* SVD of a small square upper-triangular R (c x c, f64, row-major, ld c):
 * R = W diag(s) J^T with s descending.  W and J are c x c (f64, row-major,
 * ld c).  One-sided Jacobi on the columns of R (one workgroup) gives W and s;
 * J is recovered as J_i = R^T w_i / s_i, so column i of J is accurate to about
 * u s_1 / s_i (u = 2^-53) and is zero when s_i = 0. */
int rsvd_small_svd(rsvd_handle_t handle, int32_t c, const double* R, double* s,
                   double* W, double* J, uint32_t* flags, void* work, size_t work_bytes);

#ifdef __cplusplus
}
#endif

#endif /* RSVD_MI355X_H */
