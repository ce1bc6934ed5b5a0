/*
 * rbkitk.h - C ABI of the MI355X (gfx950) implementation of randomized block
 * Krylov iteration for Tucker decomposition (rBKI-TK) and of the hierarchical
 * tensor-ring variant (rBKI-TK-TR), after Qiu, Sun, Zhou and Zhao,
 * "Towards Efficient and Accurate Approximation: Tensor Decomposition Based on
 * Randomized Block Krylov Iteration", arXiv 2211.14828.
 *
 * Conventions for every entry point
 * ---------------------------------
 * - Tensor, factor, core and workspace pointers are DEVICE pointers unless a
 *   parameter says "host".  Tensors are row-major (last index fastest).
 *   The caller owns every buffer; the library never allocates or frees caller
 *   memory, and never allocates device memory in these calls (all scratch
 *   space comes from the caller's workspace).  The one exception is
 *   rbki_server_create, which allocates the server's arena once.
 * - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *   Work is enqueued asynchronously on it; an entry point that returns a host
 *   value (rel_err, widths, a solver status) synchronises that stream before
 *   returning.  rbki_tucker, rbki_htr and the eigen-solver entry points
 *   always return the eigen-solver's status, so they always synchronise.
 * - All arguments are validated before anything is enqueued: on a status
 *   other than RBKI_OK nothing was launched, except RBKI_E_HIP (a launch or
 *   runtime error, outputs undefined) and RBKI_E_NOCONV (results written,
 *   but an eigen-solver hit its sweep limit, or the workgroups of a
 *   multi-workgroup reduction did not meet within its bounded wait).
 *   rbki_last_error() returns a thread-local message for the last failing
 *   call of the calling thread.
 * - Mode indices are 0-based; the Philox "mode" word of the sketch stream is
 *   the 0-based mode index.
 * - Thread safety: calls on different streams with disjoint buffers may run
 *   concurrently.
 */
#ifndef RBKITK_H
#define RBKITK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RBKI_OK = 0,
  RBKI_E_INVALID = 1,     /* bad argument or workspace too small; nothing launched */
  RBKI_E_NOMEM = 2,       /* reserved */
  RBKI_E_HIP = 3,         /* HIP runtime / launch error */
  RBKI_E_NOCONV = 4,      /* an eigen-solver did not finish (sweep limit, bounded wait) */
  RBKI_E_UNSUPPORTED = 5  /* valid request this build does not support */
} rbki_status;

typedef enum { RBKI_F64 = 0, RBKI_F32 = 1, RBKI_BF16 = 2 } rbki_dtype;

/* Arithmetic of the products that read the tensor (sketch, Gram/Krylov
 * products, mode products, error).  Orthonormalisation, the projected
 * eigenproblem and all norms are float64 in every form.
 *   PLAIN      : the tensor's own type (fp64 MFMA for F64, fp32 MFMA for F32,
 *                bf16 MFMA for BF16), fp32 or fp64 accumulation.
 *   MIXED_BF16 : a bf16 copy of X feeds bf16 MFMA with fp32 accumulation.
 *   MIXED_FP8  : an e4m3 copy of X with power-of-two scales per 32^N block
 *                feeds the Gram and sketch products (block-scaled fp8 MFMA,
 *                fp32 accumulation); the mode products and the error use a
 *                bf16 copy. */
typedef enum { RBKI_PLAIN = 0, RBKI_MIXED_BF16 = 1, RBKI_MIXED_FP8 = 2 } rbki_precision;

/* Subspace of each mode's factor.  RBKI_KRYLOV: the block Krylov space
 * [W, (XX^T) W, ..., (XX^T)^q W] of Alg. 1 (rBKI).  RBKI_POWER: power
 * iteration, the space of (XX^T)^q W alone, orthonormalised after every
 * step (the power-iteration comparison of Sec. 3.1, GRpi-SVD); its basis has
 * width S_n.  With q = 0 both are the single-sketch range finder (GR-SVD). */
typedef enum { RBKI_KRYLOV = 0, RBKI_POWER = 1 } rbki_variant;

/* How the modes follow each other (Alg. 2, step 6 inside the loop over n).
 * RBKI_INDEPENDENT: every factor from the original X, then the core
 * G = X x_1 U^(1)T ... x_N U^(N)T (the randomized-HOSVD form).
 * RBKI_SEQUENTIAL: sequential truncation (the ST-HOSVD form): Y_0 = X, the
 * factor of mode n from Y_{n-1}, Y_n = Y_{n-1} x_n U^(n)T, G = Y_N; mode n's
 * sketch has as many rows as Y_{n-1}'s unfolding has columns.  Modes after
 * the first read Y_{n-1} in float32 (float64 for a float64 X) in the plain
 * form, whatever `precision` says for the first. */
typedef enum { RBKI_INDEPENDENT = 0, RBKI_SEQUENTIAL = 1 } rbki_truncation;

/* Problem statement of Alg. 2: tensor order N, sizes I_n, multilinear rank
 * R_n, sketch sizes S_n = min(R_n + oversample, I_n, J_n) (Sec. 4.1 uses
 * oversample = 5), and the number of Krylov steps q ("power"; Alg. 1 gives it
 * only as Theta(log d / sqrt(eps)), Sec. 3.1 uses 2).  The Krylov basis of
 * mode n has width S'_n = min(S_n (q+1), I_n); the power variant's has width
 * S_n.
 *
 * Partial columns (Sec. 3.1): with sample_rate omega < 1 the Krylov basis of
 * mode n is built from the m_n = max(1, round(omega J_n)) sampled columns Y of
 * X_(n) instead of all J_n: W = Y Omega (Omega of m_n rows, the sketch stream
 * with J_n replaced by m_n), the Krylov steps with Y Y^T, and S_n =
 * min(R_n + oversample, I_n, m_n).  Z = Q^T X_(n) X_(n)^T Q still uses the whole
 * unfolding (Alg. 2, step 3), as do the core and the error.  The sample is
 * stratified uniform: stratum k = [floor(k J_n / m_n), floor((k+1) J_n / m_n))
 * gives the column at offset floor(w width / 2^32), w the first word of the
 * Philox block at counter (lo32(k), hi32(k), n, 1) under the sketch key. */
typedef struct {
  int order;              /* N >= 2 (N = 2 is the matrix rBKI-SVD case) */
  const int64_t *dims;    /* host[N], I_n >= 1 */
  const int64_t *ranks;   /* host[N], 1 <= R_n <= min(I_n, J_n) */
  int oversample;         /* p >= 0 */
  int power;              /* q >= 0 */
  uint64_t seed;          /* key of the Philox sketch stream */
  int precision;          /* rbki_precision */
  int variant;            /* rbki_variant (0, the Krylov space, when zero-initialised) */
  double sample_rate;     /* omega in (0, 1]: build each mode's basis from m_n = round(omega J_n)
                             columns of the unfolding (Sec. 3.1); 0 (zero-initialised) means 1 */
  int truncation;         /* rbki_truncation (0, independent modes, when zero-initialised) */
} rbki_params;

/* Library version string (static storage). */
const char *rbki_version(void);

/* Thread-local message of the last failing call ("" if none). */
const char *rbki_last_error(void);

/* ---------------------------------------------------------------------------
 * Sketch stream (Alg. 1, step 1: the Gaussian sketching matrix Omega^(n)).
 * Writes Omega^(n)T, i.e. S rows of J values, row s holding Omega^(n)[0..J-1, s]
 * = the stream values at linear indices s*J .. s*J+J-1 of (seed, mode, tag 0),
 * as `dtype` (F64: Box-Muller in double; F32 and BF16: in float, rounded).
 * out: device, S*J elements.
 */
rbki_status rbki_omega(uint64_t seed, int mode, int64_t J, int64_t S, int dtype, void *out,
                       void *stream);

/* Raw Philox4x32-10 blocks (Salmon et al., SC'11) for `count` counters:
 * ctr (device, count x 4 uint32) -> out (device, count x 4 uint32) under key
 * (seed mod 2^32, seed >> 32).  For verifying the generator bit for bit. */
rbki_status rbki_philox(const uint32_t *ctr, int64_t count, uint64_t seed, uint32_t *out, void *stream);

/* ---------------------------------------------------------------------------
 * Alg. 1 (tensor sketching via rBKI) for one mode: the orthonormal basis Q of
 * the block Krylov space span[W, (X_(n)X_(n)^T) W, ..., (X_(n)X_(n)^T)^q W],
 * W = X_(n) Omega^(n), built with orthonormalisation between steps.
 *   X      : device tensor, row-major, dims prm->dims, type xtype.
 *   mode   : n in [0, N).
 *   Qt     : device float64, S'_n x I_n row-major (row k = basis column k).
 *            Rows beyond the numerical rank of the Krylov space are zero.
 *   width  : host, receives the number of nonzero basis vectors (synchronises).
 * The unfolding is never formed: X is read through the [A_n, I_n, B_n] view,
 * X_(n)[i, a*B_n + b] = X[a, i, b] (Table 1).
 */
size_t rbki_basis_workspace(const rbki_params *prm, int xtype, int mode);
/* Rows of Qt that rbki_basis writes for this problem and mode: the basis
 * width min(S'_n, I_n) (S_n for the power variant); 0 if prm is invalid. */
int64_t rbki_basis_rows(const rbki_params *prm, int xtype, int mode);
rbki_status rbki_basis(const void *X, int xtype, const rbki_params *prm, int mode, double *Qt,
                       int64_t *width, void *workspace, size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------------------
 * Alg. 2 (rBKI-TK).  For every mode independently: Q^(n) by Alg. 1,
 * Z = Q^T X_(n) X_(n)^T Q, its eigenvectors in descending order (Remark 1),
 * U^(n) = Q Utilde(:, 1:R_n); then G = X x_1 U^(1)T ... x_N U^(N)T.
 *   core     : device, R_1 x ... x R_N row-major, out_type (F64 or F32).
 *   factors  : host array of N device pointers, factor n is I_n x R_n
 *              row-major, out_type.  Columns beyond the numerical rank of the
 *              Krylov space are zero.
 *   rel_err  : host, nullable.  ||X - [[G; U]]||_F / ||X||_F from the explicit
 *              residual, float64 accumulation (synchronises).
 */
size_t rbki_tucker_workspace(const rbki_params *prm, int xtype);
rbki_status rbki_tucker(const void *X, int xtype, const rbki_params *prm, void *core,
                        void *const *factors, int out_type, void *workspace, size_t ws_bytes,
                        double *rel_err, void *stream);

/* rbki_tucker without its final synchronisation, for callers that run
 * decompositions back to back on one stream (Alg. 2, the same work and
 * outputs as rbki_tucker, the explicit error included).  The error sums and
 * the eigen-solvers' status are copied into `result` when the stream gets
 * there; the call returns once everything is enqueued.
 *   result : host memory of rbki_tucker_result_bytes() bytes, owned by the
 *            caller.  Page-locked memory (hipHostMalloc) keeps the copy
 *            asynchronous; it must be left alone until the stream has passed
 *            this call's work.
 * Calls that share a workspace must be issued on one stream.  After the
 * stream has passed the call, rbki_tucker_result(result, &rel_err) returns
 * rel_err as rbki_tucker would, and RBKI_E_NOCONV if an eigen-solve did not
 * finish.  Invalid arguments are reported before anything is enqueued. */
size_t rbki_tucker_result_bytes(void);
rbki_status rbki_tucker_enqueue(const void *X, int xtype, const rbki_params *prm, void *core,
                                void *const *factors, int out_type, void *workspace, size_t ws_bytes,
                                void *result, void *stream);
rbki_status rbki_tucker_result(const void *result, double *rel_err);

/* rBKI-TK with the number of Krylov steps chosen by the stopping rule of
 * Sec. 4: after t = 0, 1, ... steps (every mode; the same sketch, so the
 * Krylov spaces are nested) the rank-k approximation X_t and its Fit
 * 1 - ||X - X_t||_F / ||X||_F (a fraction, against the input X, the explicit
 * residual) are formed, and the solve stops at the first t >= 1 with
 * |Fit_t - Fit_{t-1}| <= fit_tol, or at t = prm->power (the paper's 20).
 * Steps beyond ceil(I_n / S_n) cannot change a basis that spans its mode
 * space, so at most max_n ceil(I_n / S_n) steps are taken.  The outputs are
 * those of rbki_tucker with q = *q_used (bit for bit when no mode is
 * sampled).  Krylov variant, independent modes only (RBKI_E_UNSUPPORTED
 * otherwise).  Synchronises once per step.
 *   fit_tol : the Fit change that stops the iteration (the paper's 1e-3).
 *   rel_err : host, nullable: the error after the last step.
 *   q_used  : host, nullable: the number of Krylov steps taken.
 */
size_t rbki_tucker_adaptive_workspace(const rbki_params *prm, int xtype);
rbki_status rbki_tucker_adaptive(const void *X, int xtype, const rbki_params *prm, double fit_tol,
                                 void *core, void *const *factors, int out_type, void *workspace,
                                 size_t ws_bytes, double *rel_err, int *q_used, void *stream);

/* rbki_tucker for callers that cannot allocate device memory (code under
 * graph capture, tight serving loops, harnesses that forbid allocation): the
 * workspace is a fixed array of the library's own device memory instead of a
 * caller buffer.  Each device the library runs on holds one such array of
 * rbki_tucker_noalloc_limit() bytes (128 MiB) from the first load of the
 * library until the process ends; the call allocates nothing, creates no
 * stream, and runs every mode on `stream`.
 * Arguments, outputs and errors are those of rbki_tucker; a problem whose
 * workspace (rbki_tucker_workspace) exceeds the limit returns
 * RBKI_E_INVALID before anything is launched.  All calls on one device share
 * that device's array, which keeps the last call's contents: calls that
 * overlap on one device (different streams or threads) race and must not be
 * issued.  Synchronises `stream` (as rbki_tucker does). */
size_t rbki_tucker_noalloc_limit(void);
rbki_status rbki_tucker_noalloc(const void *X, int xtype, const rbki_params *prm, void *core,
                                void *const *factors, int out_type, double *rel_err, void *stream);

/* ---------------------------------------------------------------------------
 * Alg. 3 (rBKI-TK-TR) with the TR-SVD branch: rBKI-TK with the Tucker ranks
 * of prm (the compress sizes), TR-SVD of the core with TR ranks
 * (r_1, ..., r_N) and closing rank r_0 = r_N (Def. 2), then X_n = G_n x_2 U^(n).
 *   tr_ranks : host[N].
 *   tr_cores : host array of N device pointers, core n is r_{n-1} x I_n x r_n
 *              row-major, out_type.  When r_0 r_1 exceeds the rank of the
 *              first unfolding the missing directions are zero.
 *   rel_err  : host, nullable: ||X - TR(X_1..X_N)||_F / ||X||_F, from
 *              ||X - [[G;U]]||^2 + ||G - TR(G_1..G_N)||^2 (orthonormal U),
 *              both terms computed explicitly in float64 (synchronises).
 */
size_t rbki_htr_workspace(const rbki_params *prm, int xtype, const int64_t *tr_ranks);
rbki_status rbki_htr(const void *X, int xtype, const rbki_params *prm, const int64_t *tr_ranks,
                     void *const *tr_cores, int out_type, void *workspace, size_t ws_bytes,
                     double *rel_err, void *stream);

/* Alg. 3 with the TR-ALS branch named in its step 3: as rbki_htr, with TR-ALS
 * sweeps on the core instead of TR-SVD.  The cores start from the Gaussian
 * sketch stream of prm->seed with tag 2: core k's entry at linear index
 * (a S_k + i) r_k + b is z of stream (seed, k, 2) at that index, divided by
 * sqrt(S_k r_{k-1} r_k) (a zero-padded TR-SVD start would make the updates
 * rank-deficient).  Each sweep updates the
 * cores in order; core k is the least-squares fit of the core's cyclic
 * mode-k unfolding by the ring of the other cores (normal equations, minimum-
 * norm solution: eigenvalues of the Gram matrix of the design below 1e-13 of
 * the largest count as zero, so zero-padded directions stay zero).  The
 * sweeps stop when the Fit 1 - ||G - TR|| / ||G|| changes by at most fit_tol
 * (the rule of Sec. 4, 1e-3 there), or after max_sweeps (20 there).  The
 * core and the TR ranks are small: TR ranks <= 64, float64 throughout.
 *   sweeps : host, nullable: sweeps taken (synchronises once per sweep).
 */
size_t rbki_htr_als_workspace(const rbki_params *prm, int xtype, const int64_t *tr_ranks);
rbki_status rbki_htr_als(const void *X, int xtype, const rbki_params *prm, const int64_t *tr_ranks,
                         int max_sweeps, double fit_tol, void *const *tr_cores, int out_type,
                         void *workspace, size_t ws_bytes, double *rel_err, int *sweeps, void *stream);

/* ---------------------------------------------------------------------------
 * The small symmetric eigenproblem of Alg. 2, steps 3-4 (Z = Q^T X X^T Q,
 * "svd(Z)"; Remark 1): eigenvalues in descending order and unit eigenvectors
 * of a symmetric positive semidefinite float64 matrix, by one-sided Jacobi on
 * the device.
 *   Z        : device, n x n row-major (read only; must be symmetric PSD).
 *   lam      : device, n doubles, descending.
 *   Vt       : device, n x n row-major; row k is the eigenvector of lam[k],
 *              signed so that its largest-magnitude entry is positive.
 *   sweeps   : host, nullable: sweeps used (synchronises).
 * n <= 1200.  Returns RBKI_E_NOCONV if the sweep limit was reached.
 */
size_t rbki_sym_eig_workspace(int64_t n);
rbki_status rbki_sym_eig(const double *Z, int64_t n, double *lam, double *Vt, void *workspace,
                         size_t ws_bytes, int *sweeps, void *stream);

/* The k leading eigenpairs only, which is what Alg. 2, step 5 keeps (k = R_n
 * of Z's n = S (q + 1)): Householder reduction to tridiagonal form, bisection
 * on Sturm counts and inverse iteration, one workgroup per matrix.  The
 * factor step of rbki_tucker / rbki_htr uses this solver when n <= 512.
 *   Z        : device, n x n row-major (read only; only the upper triangle
 *              is read; symmetric PSD).
 *   lam      : device, k doubles, descending.
 *   Vt       : device, k x n row-major; row j is the unit eigenvector of
 *              lam[j], signed so that its largest-magnitude entry is positive.
 * 1 <= k <= n <= 512; anything else returns RBKI_E_INVALID.  For n above
 * about 165 the reduction is shared by several workgroups that wait for each
 * other with a bounded number of polls; if they do not meet, the call returns
 * RBKI_E_NOCONV (the environment variable RBKI_EIG_SPIN_LIMIT, read at each
 * call, sets that bound; 0 makes the first wait give up, for testing the
 * error path).  Synchronises the stream.
 */
size_t rbki_sym_eig_top_workspace(int64_t n, int64_t k);
rbki_status rbki_sym_eig_top(const double *Z, int64_t n, int64_t k, double *lam, double *Vt,
                             void *workspace, size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------------------
 * Serving form: a request server for many small decompositions (continuous
 * batching).  Not in the paper; it serves the same Alg. 2 decomposition
 * (rbki_tucker, with rel_err) to a stream of requests of different shapes.
 *
 * rbki_server_create allocates, once, a device arena of hbm_budget_bytes on
 * the current device and starts `slots` worker threads, each with its own
 * stream (1 <= slots <= 64).  rbki_server_submit queues a request and returns
 * at once with a ticket.  A free worker admits the oldest queued request as
 * soon as its footprint (rbki_server_request_bytes, the rbki_tucker
 * workspace) fits into the arena's free memory, and runs it on its stream;
 * requests admitted by different workers overlap on the device.  No device
 * memory is allocated after create.  The overlap is bounded by the hardware
 * queues the HIP runtime gives the process (GPU_MAX_HW_QUEUES, 4 unless set
 * before the runtime starts): streams beyond that share queues and run one
 * after the other, so set it to about `slots`.
 *   X, core, factors : device buffers as for rbki_tucker; they must stay
 *                      valid, and X unchanged, until the request is done.
 *                      X must be complete when submit is called: the
 *                      workers' streams are non-blocking and do not wait for
 *                      work on any other stream.
 *   poll             : *done = 1 once finished; then rel_err (host, nullable)
 *                      and latency_ms (host, nullable: submit to completion)
 *                      are written, the request's status is returned and the
 *                      ticket is released.  *done = 0: RBKI_OK, nothing else.
 *   wait             : blocks until done, then as poll.
 *   destroy          : finishes every submitted request, stops the workers,
 *                      frees the arena.
 * Errors: submit validates like rbki_tucker (RBKI_E_INVALID, also for a
 * footprint above the budget); a failing request reports its status
 * through poll / wait.  The server object is thread safe.
 */
typedef struct rbki_server rbki_server;
size_t rbki_server_request_bytes(const rbki_params *prm, int xtype);
rbki_status rbki_server_create(size_t hbm_budget_bytes, int slots, rbki_server **out);
rbki_status rbki_server_submit(rbki_server *server, const void *X, int xtype, const rbki_params *prm, void *core,
                               void *const *factors, int out_type, uint64_t *ticket);
rbki_status rbki_server_poll(rbki_server *server, uint64_t ticket, int *done, double *rel_err, double *latency_ms);
rbki_status rbki_server_wait(rbki_server *server, uint64_t ticket, double *rel_err, double *latency_ms);
rbki_status rbki_server_destroy(rbki_server *server);

/* Releases what the library holds between calls on its own (helper streams
 * of the concurrently running modes, events of pending timing records), after
 * the work on them has finished.  Safe to call at any time; later calls
 * recreate what they need.  Call it before the HIP runtime shuts down (the
 * Python binding registers it to run at interpreter exit). */
void rbki_release(void);

/* ---------------------------------------------------------------------------
 * Kernel timing.  When enabled, the library records HIP events around every
 * launch of the named kernels on the stream the kernel is launched on, and
 * accumulates their durations at the next synchronising call or at
 * rbki_profile_read.  Names: "gram" (Gram + sketch products), "ttm" (first
 * mode product of the core), "error" (residual reduction), "jacobi",
 * "convert", "omega".
 */
void rbki_profile_enable(int on);
void rbki_profile_reset(void);
rbki_status rbki_profile_read(const char *kernel, int64_t *launches, double *total_ms);

#ifdef __cplusplus
}
#endif
#endif /* RBKITK_H */
