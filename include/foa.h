/*
 * foa.h - C ABI of the MI355X FOA library: the modified Full Orthogonalization
 * Arnoldi (FOA) step of FOA-based streaming DMD (Anantharamu & Mahesh,
 * "A parallel and streaming Dynamic Mode Decomposition algorithm with finite
 * precision error analysis for large data").
 *
 * The state is the tuple (H, V, beta, q) of Algorithm 4: the orthonormal
 * Arnoldi basis V (n x q), the upper Hessenberg projected matrix H_bar
 * (q x (q-1)) and the upper triangular beta (q x q) with X_1^q = V beta.
 * Each push takes one snapshot psi_{q+1} through one iteration of the loop of
 * Algorithm 1: partial beta column (eq. betacolumnupdate), w = A v_q formed
 * from the snapshot (eq. avpsijp1beta), classical Gram-Schmidt with one
 * reorthogonalisation, normalisation and append, and beta completion.
 * Eigenvalues, modes, rank truncation, error indicators and coefficients
 * follow the post-processing of Algorithm 1, Algorithm 3, Section 3.2.3 and
 * Section 3.2.4.
 *
 * Conventions
 *  - Every function returns foa_status: 0 success, > 0 information,
 *    < 0 error.  Argument errors are detected before anything is enqueued.
 *  - Device memory: the caller owns every device buffer.  The library keeps
 *    its whole device state in one caller-provided workspace (at least
 *    foa_workspace_bytes() bytes, 256-byte aligned) and never allocates or
 *    frees device memory; the one device memory it holds itself is the static
 *    block workspace of foa_push_blocked_static (a fixed-size array per
 *    device).  Host scratch is library-owned and released by foa_destroy().
 *  - Streams: all device work is enqueued on the hipStream_t given to
 *    foa_init (passed as void*); calls that return device results are
 *    stream-ordered, calls that return host results synchronise the stream.
 *  - Snapshots are read-only device vectors of n entries (FP32 or FP64).  The
 *    caller keeps a snapshot valid until the stream has passed the push.
 *  - Precision: V is stored in FP64 (FOA_PREC_F64) or FP32 (FOA_PREC_F32,
 *    classical Gram-Schmidt with reorthogonalisation on an FP32 basis); all
 *    dot products, norms, H_bar, beta and the small dense linear algebra are
 *    FP64 in both forms.
 *  - A context is used by one host thread at a time.
 *  - Device-detected conditions (dependent or non-finite snapshot) are
 *    reported by the next call that synchronises (foa_sync and every call
 *    returning host data).
 */
#ifndef FOA_H
#define FOA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct foa_ctx_s *foa_ctx;
typedef struct foa_batch_s *foa_batch;

typedef enum {
  FOA_OK = 0,
  FOA_INVARIANT = 1,      /* a snapshot fell in span(V) (Section 3.2.4): the basis is
                             invariant, H_q is complete, later pushes are ignored */
  FOA_E_ARG = -1,         /* invalid argument (null pointer, size, alignment, dtype) */
  FOA_E_CAPACITY = -2,    /* push beyond the snapshot capacity n_max */
  FOA_E_STATE = -3,       /* call not valid in the current state */
  FOA_E_NONFINITE = -4,   /* a snapshot (or a quantity derived from it) was not finite;
                             it was not committed and the stream stopped */
  FOA_E_DEVICE = -5,      /* HIP runtime error */
  FOA_E_NOMEM = -6,       /* workspace or host allocation too small */
  FOA_E_NUMERIC = -7,     /* host eigen/SVD iteration did not converge */
  FOA_E_ZERO = -8         /* first snapshot has zero norm (beta_11 = 0) */
} foa_status;

typedef enum { FOA_PREC_F64 = 0, FOA_PREC_F32 = 1 } foa_prec;  /* storage of V */
typedef enum { FOA_F32 = 0, FOA_F64 = 1 } foa_dtype;

/* Largest snapshot capacity n_max the push kernels hold in registers. */
#define FOA_MAX_CAPACITY 512

/* ---- single stream ------------------------------------------------------- */

/* Workspace bytes for n rows, capacity n_max snapshots and V precision prec.
 * Host-only; does not touch the device.  FOA_E_ARG for n < 1, n_max < 1,
 * n_max > FOA_MAX_CAPACITY or an unknown prec. */
foa_status foa_workspace_bytes(int64_t n, int32_t n_max, foa_prec prec, size_t *bytes);

/* Create a context on the current HIP device.  d_workspace: device buffer of
 * ws_bytes >= foa_workspace_bytes(), 256-byte aligned, owned by the caller and
 * never freed by the library (it must outlive the context).  hip_stream:
 * hipStream_t (NULL = default stream).  breakdown_tol < 0 selects the default
 * n_max * 2^-52: a snapshot psi_{j+1} counts as dependent on its predecessors
 * when beta_{j+1,j+1} <= breakdown_tol * ||X_1^{j+1}||_F (reading of the
 * exact-arithmetic condition h_{j+1,j} = 0, Section 3.2.4).  State: q = 0. */
foa_status foa_init(foa_ctx *ctx, int64_t n, int32_t n_max, foa_prec prec, void *d_workspace,
                    size_t ws_bytes, void *hip_stream, double breakdown_tol);

/* Push one snapshot (Algorithm 4 with p = 1; for q = 0 the first-snapshot
 * normalisation of Algorithm 1, else one iteration of its loop).  d_x: device vector of n
 * entries of type x_dtype.  Asynchronous.  FOA_E_CAPACITY when q = n_max,
 * FOA_E_STATE after the stream became invariant or failed (as known to the
 * host at the last synchronising call; pushes enqueued after an undetected
 * breakdown are ignored on the device). */
foa_status foa_push_snapshot(foa_ctx ctx, const void *d_x, foa_dtype x_dtype);

/* ---- one-reduction form ---------------------------------------------------- */

typedef enum {
  FOA_FORM_CGS2 = 0,           /* Algorithm 1's order: CGS2 of w = A v_j, three sweeps per push */
  FOA_FORM_ONE_REDUCTION = 1   /* QR view with delayed reorthogonalisation: one sweep per push */
} foa_form;

/* Choose how pushes orthogonalise (before the first push: after foa_init or
 * foa_reset; FOA_E_STATE otherwise, and on a batch view).
 * FOA_FORM_ONE_REDUCTION factorises the snapshots X = V beta directly (the QR
 * view of Section 3.1) and takes H_bar from beta through eq.
 * betacolumnupdate, with the two classical Gram-Schmidt projections of
 * consecutive snapshots sharing one sweep over the basis and one global
 * reduction (delayed reorthogonalisation, Bielich et al., Parallel Computing
 * 2022) instead of the three of Algorithm 1 (the message count of Section
 * 3.2.5).  Same factors in exact arithmetic, rounding of the same
 * O(eps kappa_2) order.  With an FP32 basis the second projection is taken
 * against the stored basis's own Gram matrix (V^T V = I + E, E kept from the
 * rounding error of each finished column), which keeps the basis orthogonal
 * when a snapshot's new direction is as small as that rounding.  A column becomes final two pushes after its
 * snapshot: every synchronising call (foa_sync and the calls returning host
 * data) first finishes the pending columns (up to two sweeps; foa_flush does
 * this stream-ordered), and a dependent snapshot is found when its column
 * finishes (the stream then becomes invariant with the columns before it,
 * as in the three-sweep form).  The snapshot is copied into the basis, so the
 * caller may reuse its buffer once the stream has passed the push.  The
 * blocked form and foa_next_column are not available (FOA_E_STATE).
 * FOA_E_ARG for an FP64 basis with n_max > 257 (the sweep's register tile). */
foa_status foa_set_form(foa_ctx ctx, foa_form form);

/* One-reduction form: finish the pending columns (stream-ordered, no host
 * synchronisation); afterwards foa_copy_basis sees every snapshot taken.
 * No effect for the three-sweep form. */
foa_status foa_flush(foa_ctx ctx);

/* ---- blocked form (p snapshots per basis sweep) ---------------------------- */

/* Caller workspace of foa_push_blocked for a stream of n rows and capacity
 * n_max (about n * 32 bytes plus n_max * 32 KB). */
foa_status foa_block_workspace_bytes(int64_t n, int32_t n_max, foa_prec prec, size_t *bytes);

/* Push p snapshots (rows of d_X, row stride ld >= n elements, x_dtype) in
 * blocks of 4: the factorisation X = V beta and H_bar of the modified FOA
 * (Section 2, eq. betacolumnupdate; the QR view of Section 3.1) reached with
 * three sweeps over the basis per block instead of per snapshot, two within
 * a run of blocks (a block's last sweep also forms the next block's V^T Y
 * over the columns it sweeps).  Per block:
 * classical Gram-Schmidt of the whole block against V, twice, and a third
 * time where two passes may leave part of the block along V (a basis stored
 * in FP32 is orthonormal only to its rounding, which matters for snapshots
 * whose new directions are that small: the test compares
 * (||R2||_F / ||R1||_F) ||R2_k|| with a tenth of the basis's unit roundoff
 * times ||Z_k||), then the block's own QR by shifted CholeskyQR3 (Fukaya et
 * al., SIAM J. Sci. Comput. 2020), beta's new columns [R1 + R2 (+ R3); S] and
 * H_bar's new columns from eq. betacolumnupdate solved column by column.  The results equal the
 * sequential form's in exact arithmetic and differ by rounding of the same
 * O(eps kappa_2) order.  A block whose new diagonal entry of beta falls at or
 * under the breakdown threshold, or whose Cholesky steps fail, is taken one
 * snapshot at a time by the sequential kernels (which apply the breakdown
 * and non-finite rules), as are the first snapshot of a stream, the
 * snapshots of the call that do not fill a block (p mod 4 of them, counted
 * after that first snapshot; taken first, while the basis is smallest).  An
 * FP64 basis above 256 columns is swept in column windows of at most 256
 * (same results up to rounding order).
 * d_bws: device buffer of foa_block_workspace_bytes bytes, 256-byte aligned,
 * caller-owned, contents not preserved.  Synchronising (the host checks each
 * run of blocks).  FOA_E_CAPACITY if q + p > n_max; FOA_E_STATE on a batch
 * view or a stream that is not active; FOA_E_NOMEM for a small workspace. */
foa_status foa_push_blocked(foa_ctx ctx, const void *d_X, int64_t ld, int32_t p, foa_dtype x_dtype,
                            void *d_bws, size_t bws_bytes);

/* Size of the library's static block workspace (foa_push_blocked_static):
 * 64 MiB per device, enough for foa_block_workspace_bytes(n, n_max, prec)
 * up to about n = 1.5 million rows at n_max = 512 (about 2 million at
 * n_max = 64). */
#define FOA_BLOCK_STATIC_BYTES ((size_t)64 << 20)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): foa_push_blocked
 * with its block workspace taken from a static device array of
 * FOA_BLOCK_STATIC_BYTES that the library holds on each device it runs on
 * (until the process ends) instead of a caller buffer.  Same arguments,
 * results and errors as foa_push_blocked; allocates nothing.  FOA_E_NOMEM
 * (nothing enqueued) when foa_block_workspace_bytes(n, n_max, prec) exceeds
 * FOA_BLOCK_STATIC_BYTES; FOA_E_DEVICE if the array's device address could
 * not be looked up.  Every call on one device shares that device's array:
 * calls that overlap on one device (several contexts used from several host
 * threads, or on several streams at once) race and give wrong results; the
 * array keeps the last call's contents, and every call writes each value
 * before it reads it (the block-rejection flag is cleared by a kernel). */
foa_status foa_push_blocked_static(foa_ctx ctx, const void *d_X, int64_t ld, int32_t p, foa_dtype x_dtype);

/* In-place fill target for the next snapshot (the memory note of Appendix
 * A.1: a new snapshot may occupy storage the method already holds): *d_col receives a device buffer of n FP64 entries inside the
 * workspace (the push's work vector).  Fill it on the context's stream after
 * the previous push, then call foa_push_snapshot(ctx, *d_col, FOA_F64); the
 * first pass reads each row before it overwrites that row, so the snapshot
 * needs no storage of its own.  The contents are overwritten by every push. */
foa_status foa_next_column(foa_ctx ctx, void **d_col);

/* Push p snapshots stored as columns of a device matrix (column j at
 * d_X + j*ld elements), processed in order exactly as p single pushes
 * (Algorithm 4 with p > 1, Section 3.1). */
foa_status foa_push_block(foa_ctx ctx, const void *d_X, int64_t ld, int32_t p, foa_dtype x_dtype);

/* Wait for the stream; returns the device-side status of the pushes so far:
 * FOA_OK, FOA_INVARIANT, FOA_E_NONFINITE or FOA_E_ZERO.  q (may be NULL): basis
 * vectors held. */
foa_status foa_sync(foa_ctx ctx, int32_t *q);

/* Copy H_bar and beta to host arrays (column-major, leading dimension ld >= q+1):
 * h_Hbar gets rows 0..q (q+1 rows) of columns 0..m-1, h_beta rows/columns 0..q
 * (beta has one more column after an invariant breakdown).  m_out (may be NULL)
 * is the order of the projected matrix: q-1, or q after an invariant breakdown.
 * Either array may be NULL.  Synchronises. */
foa_status foa_get_state(foa_ctx ctx, double *h_Hbar, double *h_beta, int32_t ld, int32_t *q,
                         int32_t *m_out);

/* Write the first ncols Arnoldi vectors v_1..v_ncols (ncols <= q) into the
 * caller's device matrix d_V (n x ncols, column-major, leading dimension
 * ld >= n) in dtype.  Stream-ordered. */
foa_status foa_copy_basis(foa_ctx ctx, void *d_V, int64_t ld, foa_dtype dtype, int32_t ncols);

/* Rows [r0, r0 + nrows) of v_1..v_ncols into d_V (nrows x ncols, column-major,
 * leading dimension ld >= nrows), for streaming a basis larger than the
 * caller's scratch.  FOA_E_ARG when the row range leaves [0, n).  Stream-ordered. */
foa_status foa_copy_basis_rows(foa_ctx ctx, int64_t r0, int64_t nrows, void *d_V, int64_t ld,
                               foa_dtype dtype, int32_t ncols);

/* Rank truncation (Algorithm 1 and Algorithm 3, truncated DMD): SVD of
 * beta_m (m as in foa_get_state) on the host in FP64; r = number of singular
 * values above rel_tol * sigma_1, or, for rel_tol < 0, above
 * N * eps_s(sigma_1) (N = snapshots taken, eps_s the spacing at sigma_1 in
 * the storage precision; numerical-rank rule of Section 4.1).  r_force > 0
 * imposes r = min(r_force, m); r_force = -1 clears the truncation.  r_out and
 * h_sigma (m values, may be NULL) receive the rank and singular values.
 * Subsequent foa_modes / foa_indicators use U_r^T H_m U_r.  Synchronises. */
foa_status foa_truncate(foa_ctx ctx, double rel_tol, int32_t r_force, int32_t *r_out,
                        double *h_sigma);

/* DMD eigenvalues and modes (post-processing of Algorithm 1): eigenpairs (lambda, z)
 * of H_m (or of U_r^T H_m U_r after foa_truncate), z of unit 2-norm with the
 * entry of largest modulus real positive.  One entry per real eigenvalue and
 * per conjugate pair (its member with Im > 0), ordered by decreasing |c_j|,
 * c the coefficients of psi_1 in the mode basis (eqs. exrecon, exreconwrt).
 * Host outputs (capacity m_max entries each, any may be NULL):
 *   h_lambda 2 doubles (re, im) per entry; h_kind 0 = real, 1 = pair;
 *   h_amp |c_j|; h_err the error indicator of the entry (as foa_indicators).
 * d_phi (may be NULL): device matrix n x ncols (column-major, leading dimension
 * ld_phi >= n, dtype phi_dtype) that receives the modes V B as packed real
 * columns in entry order: one column for a real eigenvalue, two (Re, Im) for a
 * pair; ncols = entries + pairs must not exceed phi_cols (else FOA_E_ARG).
 * m_out: entries written.  Synchronises before returning host data; the mode
 * matrix is written stream-ordered. */
foa_status foa_modes(foa_ctx ctx, int32_t m_max, double *h_lambda, int8_t *h_kind, double *h_amp,
                     double *h_err, void *d_phi, int64_t ld_phi, int32_t phi_cols,
                     foa_dtype phi_dtype, int32_t *m_out);

/* Error indicators (Section 3.2.3) for every eigenpair, in the same order and
 * entry convention as foa_modes: |h_{m+1,m}| |e_m^T z| untruncated,
 * ||[(I - U_r U_r^T) H_m ; h_{m+1,m} e_m^T] U_r z||_2 truncated (0 for an
 * invariant basis).  Synchronises. */
foa_status foa_indicators(foa_ctx ctx, int32_t m_max, double *h_lambda, double *h_err,
                          int32_t *m_out);

/* Forget all snapshots (q = 0) keeping the workspace; clears truncation. */
foa_status foa_reset(foa_ctx ctx);

/* Release the context (host memory only; the workspace stays the caller's). */
foa_status foa_destroy(foa_ctx ctx);

/* Static description of a status code. */
const char *foa_status_str(foa_status s);

/* Text of the last error raised on ctx ("" if none); valid until the next call. */
const char *foa_last_error(foa_ctx ctx);

/* Tuning knobs (tests and benchmarks): "grid" (workgroups of the row passes,
 * at most 1024; 0 = automatic: all the workgroups the pass kernel of the
 * current tile width keeps resident, at least two per CU), "prefetch" (0/1: register double buffering of the next
 * panel), "nw" (0, 4, 8 or 16: wavefronts per row-pass workgroup for an FP32 basis;
 * 0 = automatic: 4 up to 128 basis columns, 8 beyond),
 * "profile" (0/1: see foa_profile).  FOA_E_ARG for an unknown key. */
foa_status foa_set_option(foa_ctx ctx, const char *key, int64_t value);

/* Timing of the row passes, enabled with foa_set_option(ctx, "profile", 1):
 * HIP events are recorded on the context's stream around every launch of the
 * fused row-pass kernels.  out[0] = launches, out[1] = their summed duration
 * in milliseconds, out[2] = their summed algorithmic bytes (per launch: the
 * j basis columns read once, plus the snapshot read by the first pass and the
 * new column written by the last), all since the previous call, which resets
 * them.  Synchronises. */
foa_status foa_profile(foa_ctx ctx, double out[3]);

/* Timing of the mode reconstruction (foa_modes with a mode matrix), enabled
 * by the same "profile" option: out[0] = launches of the reconstruction
 * kernel, out[1] = their summed duration in milliseconds, out[2] = their
 * summed algorithmic flops (2 n m r for m basis columns and r packed mode
 * columns), all since the previous call, which resets them.  Synchronises. */
foa_status foa_profile_modes(foa_ctx ctx, double out[3]);

/* ---- many independent streams (batched form) ----------------------------- */

/* Workspace for S streams with row counts n[s] and capacities n_max[s]. */
foa_status foa_batch_workspace_bytes(int32_t S, const int64_t *n, const int32_t *n_max,
                                     foa_prec prec, size_t *bytes);

/* Create S independent streams sharing one workspace and one hipStream_t.
 * Every push advances all streams by one snapshot in a single graph launch.
 * The launch configuration -- bucket launches with their row-pass grid and
 * smallest panel range per workgroup, or (FP32 basis) the persistent
 * one-launch step with its smallest range -- is chosen at init by timing each
 * candidate at 8 basis sizes spread over the run, or read from
 * tune_table_json: path of an autotuner table (read, and appended to when the
 * shape is new), or NULL to time the candidates at every init.  The
 * configuration fixes the summation order of the row passes: the same
 * configuration and the same pushes give bitwise-identical results; another
 * configuration changes them by rounding only. */
foa_status foa_batch_init(foa_batch *b, int32_t S, const int64_t *n, const int32_t *n_max,
                          foa_prec prec, void *d_workspace, size_t ws_bytes, void *hip_stream,
                          double breakdown_tol, const char *tune_table_json);

/* Advance every stream by one snapshot.  d_x_ptrs: DEVICE array of S device
 * pointers (FP32 or FP64 per x_dtype); a NULL entry leaves that stream idle.
 * Asynchronous (one hipGraphLaunch; the graph leaves out the tile buckets no
 * stream can occupy yet, one graph per widest bucket, captured on first use). */
foa_status foa_batch_push(foa_batch b, const void *const *d_x_ptrs, foa_dtype x_dtype);

/* Wait; h_q / h_status (may be NULL) receive per-stream q and status.
 * FOA_E_DEVICE also when the persistent step reported that one of its bounded
 * waits ran out or that a group of its workgroups did not complete (the
 * bound, 2^22 polls, can be lowered for tests with the environment variable
 * FOA_PERSIST_SPIN, read at foa_batch_init). */
foa_status foa_batch_sync(foa_batch b, int32_t *h_q, int32_t *h_status);

/* Context view of stream s for get_state / copy_basis / truncate / modes /
 * indicators.  The view is owned by the batch (do not destroy it); pushes go
 * through foa_batch_push only (FOA_E_STATE otherwise). */
foa_status foa_batch_view(foa_batch b, int32_t s, foa_ctx *view);

/* Choose the form of every stream of the batch (before the first push: after
 * foa_batch_init or foa_batch_reset; FOA_E_STATE otherwise), as foa_set_form
 * does for one stream.  FOA_FORM_ONE_REDUCTION: each step runs one sweep per
 * tile bucket over the planned ranges, then every stream's reduction, H_bar
 * product and finalize (one graph launch per step); the launch configuration
 * is tuned again for it (table key with "/form1").  foa_batch_sync first
 * finishes every stream's pending columns (two flush steps); views show the
 * state as of the last foa_batch_sync.  FOA_E_ARG for an FP64 basis with a
 * capacity above 257. */
foa_status foa_batch_set_form(foa_batch b, foa_form form);

/* One-reduction form: enqueue the two flush steps that finish every stream's
 * pending columns (the same steps foa_batch_sync runs first), without waiting;
 * nothing to do when no push came since the last flush, and for the CGS2
 * form.  Stream-ordered; a later foa_batch_push continues the streams. */
foa_status foa_batch_flush(foa_batch b);

/* Forget all snapshots of every stream (q = 0), keeping workspace, tuning and
 * graphs.  Stream-ordered. */
foa_status foa_batch_reset(foa_batch b);

foa_status foa_batch_destroy(foa_batch b);

#ifdef __cplusplus
}
#endif

#endif /* FOA_H */
