/*
 * gmgm.h -- C ABI of the MI355X (gfx950) hot path of the multi-axis
 * Kronecker-sum Gaussian graphical model (arXiv 2407.19892, "Making
 * Multi-Axis Gaussian Graphical Models Scalable to Millions of Cells").
 *
 * Conventions for every entry point:
 *   - Array arguments are DEVICE pointers owned by the caller unless marked
 *     "host".  The library never frees caller memory.  It owns only its
 *     workspace, held in the context and released by gmgm_destroy.
 *   - Work is enqueued on the context's HIP stream and the call returns
 *     without waiting, except where a call is marked "synchronises".
 *   - No exception crosses the ABI.  Each call returns a gmgm_status; the
 *     context keeps a message for the last failure (gmgm_last_error).
 *     Argument and shape checks happen before anything is launched; on such
 *     an error nothing is enqueued and outputs are untouched.
 *   - Faults found on the device (non-finite inputs, HIP errors) are reported
 *     by the next synchronising call (gmgm_sync or a call that synchronises).
 *   - One context per host thread and stream.  Calls on one context must not
 *     overlap.
 */
#ifndef GMGM_H
#define GMGM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gmgm_ctx* gmgm_ctx_t;

typedef enum {
  GMGM_OK = 0,
  GMGM_E_ARG = 1,      /* null pointer, bad enum, out-of-range scalar */
  GMGM_E_SHAPE = 2,    /* inconsistent sizes */
  GMGM_E_DOMAIN = 3,   /* non-finite or non-positive input where positive finite is required */
  GMGM_E_NOCONV = 4,   /* iterative solve hit its iteration limit */
  GMGM_E_OVERFLOW = 5, /* a fixed-capacity device buffer overflowed */
  GMGM_E_HIP = 6,      /* HIP runtime or library failure */
  GMGM_E_NOMEM = 7     /* device allocation failed */
} gmgm_status;

typedef enum {
  GMGM_FP32 = 0,      /* FP32 operands, FP32 MFMA (32x32x2) */
  GMGM_BF16 = 1,      /* BF16 operands, FP32 accumulation (32x32x16) */
  GMGM_FP8_E4M3 = 2   /* OCP FP8 e4m3 operands with power-of-two row/tile scales,
                         FP32 accumulation (32x32x64 f8f6f4) */
} gmgm_prec;

/* Version of this ABI (major * 10000 + minor * 100 + patch). */
int gmgm_version(void);

/* Create a context on HIP device `device` that enqueues on `hip_stream`
 * (a hipStream_t; NULL means the legacy default stream).  Synchronises. */
gmgm_status gmgm_create(gmgm_ctx_t* ctx, int device, void* hip_stream);

/* Release the context and its workspace.  Synchronises.  NULL is ignored. */
void gmgm_destroy(gmgm_ctx_t ctx);

/* Change the stream later calls enqueue on. */
gmgm_status gmgm_set_stream(gmgm_ctx_t ctx, void* hip_stream);

/* Message of the last failed call on this context ("" if none).  The string
 * is owned by the context and valid until the next call on it. */
const char* gmgm_last_error(gmgm_ctx_t ctx);

/* Wait for all work enqueued by this context and report the first device-side
 * fault recorded since the previous gmgm_sync (GMGM_E_DOMAIN for non-finite
 * inputs found by a kernel, GMGM_E_HIP for runtime errors).  Synchronises. */
gmgm_status gmgm_sync(gmgm_ctx_t ctx);

/* Enable (1) or disable (0) HIP-event timing of each call's dominant kernel
 * (the MFMA sweep of gmgm_recompose_topk), recorded on the context stream. */
gmgm_status gmgm_set_timing(gmgm_ctx_t ctx, int enable);

/* Total duration (ms, host) and count (host) of the timed kernels recorded
 * since the previous query; clears the record.  Synchronises. */
gmgm_status gmgm_kernel_times(gmgm_ctx_t ctx, double* total_ms, int64_t* count);

/* Counters of one gmgm_recompose_topk call (filled only when requested). */
typedef struct {
  int64_t cand_total;       /* candidates (approximate top-C entries) kept by the sweep */
  int64_t rows_fallback;    /* rows the first sweep could not certify (re-swept) */
  int64_t rows_near_tie;    /* certified rows whose k-th and (k+1)-th exact |Psi| differ
                               by < 1e-6 relative */
  int64_t rows_exact;       /* rows the re-sweep could not certify either (exact
                               FP64 scan of the whole row) */
  double mfma_flops;        /* MFMA flops executed by the sweeps (padded K) */
  int64_t symmetric;        /* 1: the first sweep ran in the symmetric form (BF16,
                               every row of a large Psi); 0: the full sweep */
} gmgm_topk_stats;

/*
 * Fused eigen-recomposition with per-row top-k thresholding into CSR.
 *
 * Algorithm 1, final loop ("threshold simultaneously with recomposition"),
 * with the per-row strongest-edge rule of the experiments: for each row i in
 * [row_begin, row_end) of Psi = V diag(psi) V^T,
 *   keep the k columns j != i with the largest |Psi_ij| (ties to smaller j),
 * without forming Psi.
 *
 *   n, r        V is n x r, row-major FP32 (device).  2 <= n <= 2^31 - 64,
 *               1 <= r <= 32768.
 *   psi         r FP64 eigenvalues (device).
 *   row_begin, row_end   0 <= row_begin < row_end <= n.
 *   k           1 <= k <= 64 and k <= n - 1.
 *   prec        operand precision of the first MFMA sweep (gmgm_prec).  Every
 *               precision ends the same way: candidates are rescored exactly
 *               (FP64 from the FP32 V and FP64 psi); rows whose rounding
 *               margin cannot certify the candidate set are re-swept (r <= 128
 *               and k <= 24: FP32 operands after an FP32 sweep, else each
 *               FP32 operand split into two BF16 parts hi + lo with
 *               hi*hi + hi*lo + lo*hi formed on the matrix cores; otherwise
 *               FP32 operands), and rows that still fail are scanned exactly
 *               in FP64, so the output does not depend on `prec`.
 *   cand_cap    length of the sweep's per-lane candidate lists; must exceed k.
 *               r <= 128 and k <= 24 (W held in registers through the sweep):
 *               16 or 32, 0 picks 32 for BF16 / FP8 (a list covers a whole
 *               row) and 16 for FP32 (half a row).  Otherwise (the contraction
 *               streamed in chunks of 32; FP8 requests run with BF16
 *               operands, and every request with FP32 operands when r > 4096,
 *               where the BF16 bound certifies no row): 32, 64 or 128, 0
 *               picks the smallest that is at least 2k.
 *   row_ptr_out (row_end - row_begin + 1) int64: row_ptr[t] = k * t.
 *   col_out     k * (row_end - row_begin) int32, ascending within a row.
 *   val_out     k * (row_end - row_begin) FP32: Psi_ij (signed), rounded
 *               from the FP64 rescoring.
 *   stats       host pointer or NULL; filled when non-NULL.
 * Symmetric form (Psi = Psi^T; the computational-complexity appendix counts
 * each pair once): a BF16 call for every row (row_begin = 0, row_end = n,
 * r <= 128, k <= 24) with n >= 800000 (or n >= 1024 and the environment
 * variable GMGM_RECOMPOSE_PATH=symmetric; =full turns it off) computes only
 * the 32 x 32 tiles on or above the diagonal band of 512-row blocks.  Each
 * row's list then starts from a bound taken from a sweep over every 8th
 * column tile (the exact k-th of that sample's top k, less the row's
 * rounding margin), and every value of a computed tile above the bound of
 * its column's row is kept for that row too.  Same results, same certificate
 * (a row also certifies only when its bound plus margin is below its exact
 * k-th value); when the kept values outgrow their pool (or one wave keeps
 * more in one stage of a few column tiles than eight times the number
 * expected) the call runs the full sweep instead (stats->symmetric = 0).
 * At n = 10^6, r = 100, k = 10 it executes 0.60 of the full sweep's MFMA
 * work in about 0.92 of its time; below about 8e5 rows its bound pass and
 * grouping cost more than the skipped tiles save.
 * The call synchronises once after the first sweep (and once more when rows
 * need the re-sweep) to size the re-sweep of uncertified rows.  With
 * the contraction streamed, rows the FP32 sweep cannot certify get their
 * exact FP64 values in row panels (at most 256 MiB of workspace each).
 * Non-finite V or psi are reported as GMGM_E_DOMAIN by the next
 * synchronising call (the outputs are then undefined).
 */
gmgm_status gmgm_recompose_topk(gmgm_ctx_t ctx, int64_t n, int64_t r, const float* V,
                                const double* psi, int64_t row_begin, int64_t row_end,
                                int32_t k, gmgm_prec prec, int32_t cand_cap,
                                int64_t* row_ptr_out, int32_t* col_out, float* val_out,
                                gmgm_topk_stats* stats);

/*
 * gmgm_recompose_topk for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same arguments, checks and results, with every workspace
 * buffer carved from a fixed device array of 128 MiB that the library holds
 * on each device from its load until the process ends (its address is looked
 * up when a context is created on the device).  Nothing is allocated: no
 * hipMalloc or hipFree, no library routine that allocates, no timing events
 * (gmgm_set_timing does not record this call).  The first sweep's workspace
 * (V and W repacked, row norms, candidate lists) must fit: the column splits
 * are reduced until it does, and a call whose workspace still exceeds the
 * array is rejected with GMGM_E_SHAPE before anything is launched (BF16,
 * r = 100: n = 100000 fits, n = 1000000 does not).  Rows the first sweep
 * cannot certify are re-swept (as above) when that sweep's buffers fit in what
 * is left of the array, else scanned exactly (the result is the same).  Every
 * call on a device shares that device's array, which keeps the last call's
 * contents (what must start at zero is cleared by each call): calls that
 * overlap on one device, from any context or stream, race.  Synchronises as
 * gmgm_recompose_topk does.
 */
gmgm_status gmgm_recompose_topk_noalloc(gmgm_ctx_t ctx, int64_t n, int64_t r, const float* V,
                                        const double* psi, int64_t row_begin, int64_t row_end,
                                        int32_t k, gmgm_prec prec, int32_t cand_cap,
                                        int64_t* row_ptr_out, int32_t* col_out, float* val_out,
                                        gmgm_topk_stats* stats);

/*
 * The rounding constant c of the certificate that makes every operand
 * precision of gmgm_recompose_topk / gmgm_recompose_threshold exact
 * (Algorithm 1, final loop, read as an exact per-row selection): with W = V
 * diag(psi), the sweep's approximate value of Psi_ij = W_i . V_j satisfies
 *   |Psi~_ij - Psi_ij| <= beta_i = c ||W_i||_2 max_j ||V_j||_2,
 * from the operand format's unit roundoff (FP32 2^-24, BF16 2^-8, FP8 e4m3
 * 2^-4 plus its subnormal floor; W is rounded to FP32 first), one FP32 ulp per
 * accumulation step over the padded depth, and Cauchy-Schwarz.
 *   prec        gmgm_prec value.
 *   r           the rank, 1 <= r <= 32768.
 *   c_out       host double: c.
 *   kpad_out    host int32 or NULL: the padded MFMA depth for r (r > 128:
 *               the streamed sweep's, a multiple of 32, with FP8 requests
 *               reported for their BF16 operands and every request above
 *               r = 4096 for FP32 operands, as the sweep runs them).
 * Host arithmetic only (no context, no device).  GMGM_E_ARG / GMGM_E_SHAPE
 * for a bad precision or rank.
 */
gmgm_status gmgm_rounding_bound(int32_t prec, int64_t r, double* c_out, int32_t* kpad_out);

/*
 * Fused eigen-recomposition with a fixed threshold into CSR: the significance
 * rule of Theorem 3 (keep the statistically significant edges), or any fixed
 * threshold.  For each row i in [row_begin, row_end) of Psi = V diag(psi) V^T,
 *   keep every column j != i with |Psi_ij| >= thr, in ascending j,
 * without forming Psi.
 *
 *   n, r, V, psi, row_begin, row_end, prec   as gmgm_recompose_topk.
 *   thr         the threshold, positive and finite (GMGM_E_DOMAIN otherwise).
 *   max_per_row > 0: a row keeping more entries is an error (GMGM_E_OVERFLOW);
 *               <= 0: no limit.
 *   row_ptr_out (row_end - row_begin + 1) int64 (device), always written.
 *   col_out, val_out   `capacity` int32 / FP32 entries (device); Psi_ij
 *               (signed) rounded from the FP64 value.
 *   capacity    room in col_out / val_out (>= 0); the call also uses this
 *               many entries of workspace.
 *   nnz_out     host int64: the number of kept entries.
 * The MFMA sweep in `prec` keeps every value within the row's rounding bound
 * of the threshold (up to 1024 per row); these candidates are decided exactly
 * in FP64, and rows with more candidates are scanned exactly, so the output
 * does not depend on `prec`.  When the total exceeds `capacity` the call
 * returns GMGM_E_OVERFLOW with *nnz_out and row_ptr_out holding the true
 * sizes, so that the caller can size the output and call again.
 * GMGM_E_DOMAIN for non-finite V or psi.  Synchronises.
 */
gmgm_status gmgm_recompose_threshold(gmgm_ctx_t ctx, int64_t n, int64_t r, const float* V,
                                     const double* psi, int64_t row_begin, int64_t row_end,
                                     double thr, gmgm_prec prec, int32_t max_per_row,
                                     int64_t* row_ptr_out, int32_t* col_out, float* val_out,
                                     int64_t capacity, int64_t* nnz_out);

/*
 * The significance threshold of Theorem 3 for axis l (host computation).
 * Under the null hypothesis that modality gamma has precision sigma_gamma^-2 I,
 * an edge psi_lij is asymptotically N(0, 4 d_l / sum_gamma d^gamma_all
 * sigma_gamma^4), the sum over the n_mod modalities that contain axis l; the
 * two-sided Bonferroni test at level alpha over n_tests edges keeps
 *   |psi_lij| >= 2 z sqrt(d_l / sum_gamma d^gamma_all sigma_gamma^4),
 *   z = Phi^-1(1 - alpha / (2 n_tests)).
 *
 *   d_l         size of axis l (>= 2).
 *   n_mod       number of modalities containing axis l (>= 1).
 *   d_all       n_mod host doubles: d^gamma_all, the product of the modality's
 *               axis sizes.
 *   trace_s     n_mod host doubles: tr(S^gamma), the modality's sum of squared
 *               entries; sigma_gamma^2 = trace_s / d_all (the null model's
 *               maximum-likelihood variance).
 *   alpha       test level in (0, 1).
 *   n_tests     Bonferroni count; <= 0 selects d_l (d_l - 1) / 2.
 *   thr_out     host double.
 * No device work; ctx may be NULL (errors are then returned without a
 * message).
 */
gmgm_status gmgm_significance_threshold(gmgm_ctx_t ctx, int64_t d_l, int32_t n_mod, const double* d_all,
                                        const double* trace_s, double alpha, double n_tests,
                                        double* thr_out);

/*
 * Small-axis Gram matrix G = X^T X (problem setup: S_l = mat_l[D] mat_l[D]^T,
 * formed only for the small axis; no centring or scaling).
 *
 *   n, p        X is n x p (cells x genes); 1 <= p <= 65536.
 *   nnz         number of stored entries.
 *   row_ptr     n + 1 int64 (device), row_ptr[0] = 0, non-decreasing, <= nnz.
 *   col         nnz int32 column indices in [0, p) (device).  Duplicates add up.
 *   val         nnz FP32 values (device), or NULL for all ones (binary data).
 *   G           p x p FP32 output, row-major (device); exactly symmetric.
 * Two paths, picked from (n, p, nnz) without synchronising (the environment
 * variable GMGM_GRAM_PATH=dense or =sparse forces one):
 *   sparse  the products of each row's nonzeros, added in FP64 into 128 x 128
 *           tiles (the input-sparsity appendix: X is never densified).  The
 *           nonzeros are first copied block-major (nnz x 5 bytes); rows whose
 *           columns are not strictly increasing take a slower exact route.
 *           Workspace: the copy, per-row block offsets (<= 2 GiB per row
 *           chunk) and FP64 partials (p_pad^2 x splits, p_pad = p rounded up
 *           to 128).  Result order-dependent in the last FP64 bits only.
 *   dense   row panels densified (<= 2 GiB), FP32 MFMA products accumulated
 *           in FP32 over at most 2048 rows, then in FP64; partials p_pad^2 x
 *           splits (<= 8 GiB, p_pad = p rounded up to 256).  Deterministic
 *           for CSR input without duplicate columns.
 * Malformed CSR is reported as GMGM_E_SHAPE and non-finite values as
 * GMGM_E_DOMAIN by the next synchronising call; asynchronous otherwise.
 */
gmgm_status gmgm_gram(gmgm_ctx_t ctx, int64_t n, int64_t p, int64_t nnz, const int64_t* row_ptr,
                      const int32_t* col, const float* val, float* G);

/*
 * FP64 eigendecomposition of the symmetric Gram (Algorithm 1, first loop;
 * Theorem 1 makes these eigenvectors the MLE's).
 *
 *   p           1 <= p <= 46340.
 *   G           p x p FP32 symmetric (device, row-major); its upper triangle
 *               (row <= column) is read.
 *   evals       p FP64 (device), descending.
 *   evecs       p x p FP64 (device), column-major: column j (evecs[j p .. j p + p))
 *               is the unit eigenvector of evals[j]; NULL computes the
 *               eigenvalues only (faster: no back-transformation).
 *   rank_out    host, or NULL: numerical rank #{j : evals[j] > p 2^-52 evals[0]}.
 * Uses rocSOLVER's divide-and-conquer solver on an FP64 copy.  Synchronises.
 * GMGM_E_DOMAIN for non-finite G, GMGM_E_NOCONV if the solver reports failure.
 */
gmgm_status gmgm_eigh_small(gmgm_ctx_t ctx, int64_t p, const float* G, double* evals, double* evecs,
                            int64_t* rank_out);

/*
 * Cell-axis factor ("top r left singular vectors" of X, Algorithm 1 first
 * loop) through the exact identity U = X V[:, :r] diag(e[:r])^(-1/2).
 *
 *   n, p, nnz, row_ptr, col, val   X in CSR as for gmgm_gram.
 *   evecs       column-major FP64 eigenvectors (device), column j at
 *               evecs + j ldv; ldv >= p.
 *   evals       >= r positive FP64 eigenvalues (device).
 *   r           1 <= r <= min(p, 256).
 *   U           n x r FP32 output, row-major (device).
 * FP64 accumulation of FP32 X times the FP32-rounded scaled eigenvectors.
 * Asynchronous; malformed CSR -> GMGM_E_SHAPE, non-finite or non-positive
 * eigenvalues / non-finite values -> GMGM_E_DOMAIN at the next synchronising call.
 */
gmgm_status gmgm_sketch(gmgm_ctx_t ctx, int64_t n, int64_t p, int64_t nnz, const int64_t* row_ptr,
                        const int32_t* col, const float* val, const double* evecs, int64_t ldv,
                        const double* evals, int64_t r, float* U);

/*
 * Nonparanormal Skeptic of a sparse matrix, kept sparse ("Preserving input
 * sparsity": the rank-based Gaussian copula transform used before the Gram in
 * the paper's real-data runs).  Every column g of the n x p CSR matrix X
 * (cells x genes) is transformed marginally across its n entries, implicit
 * zeros included:
 *   f(x) = Phi^-1(rank(x) / (n + 1)),  rank(x) = 1 + #{entries of the column below x}
 * (ties share the smallest rank).  All zeros of a column map to z_g, so the
 * transformed matrix is S + 1 z^T with S of X's sparsity pattern.
 *
 *   n, p, nnz, row_ptr, col, val   X as in gmgm_gram (val NULL: all ones);
 *               nnz < 2^32.
 *   val_out     nnz FP32 (device): S at X's entries, f(x_ig) - z_g (0 where
 *               x_ig = 0), in X's entry order.
 *   z_out       p FP64 (device): z_g = f(0) of column g.
 *   csum_out    p FP64 (device): column sums of S (for gmgm_gram_shifted).
 * Synchronises once (malformed CSR -> GMGM_E_SHAPE, non-finite values ->
 * GMGM_E_DOMAIN before anything is sorted).  Uses rocPRIM's segmented radix
 * sort for the per-column ordering.
 */
gmgm_status gmgm_skeptic(gmgm_ctx_t ctx, int64_t n, int64_t p, int64_t nnz, const int64_t* row_ptr,
                         const int32_t* col, const float* val, float* val_out, double* z_out,
                         double* csum_out);

/*
 * Gram of X + 1 z^T (the transformed matrix of gmgm_skeptic) from X's CSR:
 *   G = X^T X + c z^T + z c^T + n z z^T,  c = X^T 1 (csum),
 * the rank-two correction added in FP64 before rounding.  Arguments as
 * gmgm_gram, plus z and csum (p FP64 each, device).
 */
gmgm_status gmgm_gram_shifted(gmgm_ctx_t ctx, int64_t n, int64_t p, int64_t nnz, const int64_t* row_ptr,
                              const int32_t* col, const float* val, const double* z, const double* csum,
                              float* G);

/*
 * Cell factor of X + 1 z^T: U = (X + 1 z^T) V[:, :r] diag(e)^-1/2, i.e.
 * gmgm_sketch's X V diag(e)^-1/2 plus the row z^T V[:, :r] diag(e)^-1/2 on
 * every row.  Arguments as gmgm_sketch, plus z (p FP64, device).
 */
gmgm_status gmgm_sketch_shifted(gmgm_ctx_t ctx, int64_t n, int64_t p, int64_t nnz, const int64_t* row_ptr,
                                const int32_t* col, const float* val, const double* evecs, int64_t ldv,
                                const double* evals, int64_t r, const double* z, float* U);

/* A CSR matrix (all arrays device, caller-owned): row_ptr has n_rows + 1
 * int64 entries, col and val nnz entries; val NULL means all ones. */
typedef struct {
  int64_t n_rows, n_cols, nnz;
  const int64_t* row_ptr;
  const int32_t* col;
  const float* val;
} gmgm_csr;

/* X^T in CSR form (the CSC of X): row_ptr_t (n_cols + 1 int64), col_t (nnz
 * int32 row indices of X), val_t (nnz FP32; ones when X.val is NULL).  The
 * order of entries within a transposed row is not fixed.  Asynchronous;
 * malformed X is reported as GMGM_E_SHAPE by the next synchronising call. */
gmgm_status gmgm_csr_transpose(gmgm_ctx_t ctx, gmgm_csr X, int64_t* row_ptr_t, int32_t* col_t, float* val_t);

/*
 * Leading eigenpairs of S = D D^T for an axis shared by several modalities,
 * D = [X_1 | ... | X_B] (the Notation section's concatenation; S's
 * eigenvectors are D's left singular vectors, Algorithm 1's first loop), by
 * randomized subspace iteration (Halko, Martinsson and Tropp 2011):
 *   Y = D Omega; Q = orth(Y); q times { Q' = orth(D^T Q); Q = orth(D Q') };
 *   Z = D^T Q; Z^T Z = W diag(theta) W^T (theta descending);
 *   evals = theta[:r], vecs = Q W[:, :r].
 * orth() is the thin-QR Q factor with a positive R diagonal (CholeskyQR2).
 *
 *   n_blocks    1..16 blocks X_m, each n x p_m (same n).
 *   blocks      host array of the X_m; blocks_t: host array of their
 *               transposes (p_m x n, e.g. from gmgm_csr_transpose).
 *   omega       (sum p_m) x k FP64 row-major test matrix (device).
 *   k           subspace width, 1..128, k <= min(n, sum p_m); q: 0..64.
 *   r           1..k eigenpairs returned.
 *   evals       r FP64 (device), descending.
 *   vecs        n x r FP32 row-major (device), orthonormal columns.
 * Sparse products are this library's FP64-accumulating kernels; the k-wide
 * dense steps use rocBLAS (dgemm, dtrsm) and rocSOLVER (dpotrf, dsyevd).
 * Synchronises.  GMGM_E_NOCONV if a basis is numerically rank deficient.
 */
gmgm_status gmgm_subspace_eig(gmgm_ctx_t ctx, int32_t n_blocks, const gmgm_csr* blocks,
                              const gmgm_csr* blocks_t, const double* omega, int64_t k, int32_t q,
                              int64_t r, double* evals, float* vecs);

/* Result of one gmgm_solve_eigs call. */
typedef struct {
  int32_t iterations;       /* Newton iterations taken */
  int32_t converged;        /* 1 if the KKT residual reached tol */
  int32_t n_flat;           /* number of zero-slope shift directions fixed by the gauge rule */
  int32_t warm_used;        /* 1 if the warm start was used (its NLL was not above 1/E's) */
  double kkt;               /* final scaled KKT residual */
  int64_t n_pinned[8];      /* per axis: eigenvalues that end at their bound eps_l */
  double eps[8];            /* per axis: the bound used */
} gmgm_solve_info;

/*
 * Eigenvalue maximum-likelihood estimate (Algorithm 1's eigenvalue loop;
 * eigenvalue-gradient Proposition; Existence lemma).  With the eigenvectors
 * fixed by Theorem 1, minimise over lambda_l,i >= eps_l
 *   NLL = 1/2 [ sum_l sum_i E_l,i lambda_l,i
 *               - sum_{modalities (a,b)} sum_{i<r_a, j<r_b} log(lambda_a,i + lambda_b,j) ].
 * Projected Newton (Schur complement on a minimum-rank vertex cover of the
 * modality graph, Cholesky of that system on the device), Armijo search, FP64
 * throughout, deterministic reductions.  Start: Algorithm 1's 1/E, or `warm`.
 * Shift directions along which the NLL is flat (every modality's two axes
 * shifted by +c and -c with equal traces) are fixed to the gauge of 1/E.  A
 * warm start is moved to that gauge, clipped to the box, and used only when
 * its NLL is not above that of 1/E.  Per iteration a free eigenvalue may
 * shrink by at most a factor 64.  After 30 iterations the step rule switches
 * to an escape mode (active set: coordinates whose diagonal step, with the
 * Levenberg-Marquardt diagonal h + |g|/lambda, reaches the bound; no shrink
 * limit), which reaches minimisers on the box along directions of almost zero
 * slope (axes whose traces agree only to rounding).
 *
 *   n_axes       2..8 axes.
 *   ranks        host, n_axes retained ranks r_l >= 1.
 *   E            host array of n_axes device pointers; E[l] holds r_l positive
 *                finite FP64 eigenvalues of S_l (any order).
 *   n_mod        1 .. n_axes (n_axes - 1) / 2 modalities.
 *   modalities   host, 2 * n_mod axis indices (a, b), a != b, pairs distinct;
 *                every axis must belong to one.
 *   eps          host, n_axes positive bounds, or NULL for 1e-10 / max_i E_l,i.
 *   warm         host array of n_axes device pointers (finite starting
 *                eigenvalues; moved to the gauge, then clipped to the box), or NULL.
 *   tol          stop when max over coordinates of |g| / (E/2) (free) or
 *                max(0, -g) / (E/2) (at the bound) is <= tol; 1e-12 is typical.
 *   max_iter     Newton iteration limit (>= 0).
 *   lambda_out   host array of n_axes device pointers, r_l FP64 each (written).
 *   info         host pointer or NULL.
 * The Schur system (sum of the hub axes' ranks) is limited to 32768 unknowns
 * (factorised by one workgroup up to 2048, by rocSOLVER's Cholesky above;
 * its nS^2 FP64 entries are workspace).
 * Synchronises (every iteration reads scalars back).  Returns GMGM_E_NOCONV
 * (outputs written, info filled) when tol is not reached in max_iter
 * iterations or the line search stalls; GMGM_E_DOMAIN for non-positive or
 * non-finite E, non-finite warm starts or bad eps.
 */
gmgm_status gmgm_solve_eigs(gmgm_ctx_t ctx, int32_t n_axes, const int64_t* ranks,
                            const double* const* E, int32_t n_mod, const int32_t* modalities,
                            const double* eps, const double* const* warm, double tol,
                            int32_t max_iter, double* const* lambda_out, gmgm_solve_info* info);

/*
 * Eigenvalue maximum-likelihood estimate for modalities of any number of axes
 * (tensor-variate data; the model equation with the Kronecker sum of K >= 2
 * axes, whose eigenvalues are the sums lambda_{l_1,i_1} + ... + lambda_{l_K,i_K}
 * over all index tuples; eigenvalue-gradient Proposition; Existence lemma):
 * minimise over lambda_l,i >= eps_l
 *   NLL = 1/2 [ sum_l sum_i E_l,i lambda_l,i
 *               - sum_{modalities} sum_{index tuples} log(sum of the tuple's lambdas) ].
 * Same method, start, gauge rule, stopping rule and record as gmgm_solve_eigs
 * (the record's per-axis arrays cover axes 0..7); the Newton system is held
 * dense over all sum_l r_l coordinates (the Hessian couples every two axes of a
 * modality through sums over the others) and solved by eliminating each
 * modality's private axes (those in no other modality) before the shared ones,
 * FP64, deterministic reductions; the same escape mode after 30 iterations
 * (modalities whose traces agree only to the rounding of FP32 Grams).  With
 * every modality of two axes the solution is that of gmgm_solve_eigs.
 *
 *   n_axes       2 .. 64 axes.
 *   ranks, E, eps, warm, tol, max_iter, lambda_out, info: as for
 *                gmgm_solve_eigs (host arrays of n_axes entries).
 *   n_mod        1 .. 64 modalities.
 *   mod_len      host, n_mod axis counts K_t, 2 <= K_t <= min(n_axes, 8).
 *   mod_axes     host, sum_t K_t axis indices: modality t's distinct axes,
 *                modalities one after another.  No two modalities may have the
 *                same axis set; every axis must belong to one.
 * Limits: sum_l r_l <= 8192 (the system is held dense: 8 (sum_l r_l)^2 bytes
 * of workspace); per modality at most 2^40 index tuples, the product of any
 * K - 1 of its ranks at most 2^32 and of any K - 2 at most 2^26 (the work of
 * one wave and of one cross-block thread); GMGM_E_SHAPE otherwise.  Each
 * iteration costs about K (K + 1) / 2 passes over the tuples in FP64
 * divisions, plus a pass of logarithms per line-search trial.  Synchronises.  Returns GMGM_E_NOCONV (outputs
 * written, info filled) when tol is not reached; GMGM_E_DOMAIN for
 * non-positive or non-finite E, non-finite warm starts or bad eps.
 */
gmgm_status gmgm_solve_eigs_tensor(gmgm_ctx_t ctx, int32_t n_axes, const int64_t* ranks,
                                   const double* const* E, int32_t n_mod, const int32_t* mod_len,
                                   const int32_t* mod_axes, const double* eps,
                                   const double* const* warm, double tol, int32_t max_iter,
                                   double* const* lambda_out, gmgm_solve_info* info);

/*
 * Learned warm start of the eigenvalue MLE: a small network predicts the
 * solution from the two axes' spectra and replaces Algorithm 1's start
 * lambda^0 = 1/E (gmgm_solve_eigs then finishes from it; its result does not
 * depend on the start).  The paper fixes no network; this one is:
 *   features (1028 FP32): each axis' log-spectrum resampled to 512 bins at the
 *     0-based fractional indices t_b = (b + 1/2) r / 512 - 1/2 (clamped to
 *     [0, r-1], linear interpolation), both shifted by max(log E_c[0], log E_g[0]),
 *     then log r_c, log r_g, log d_c, log d_g;
 *   network: 1028 -> 256 -> 256 -> 1024, SiLU after the hidden layers;
 *     parameters are one FP32 vector W1 (256x1028), b1, W2 (256x256), b2,
 *     W3 (1024x256), b3, row-major, gmgm_ws_param_count() floats;
 *   outputs (1024 FP32): two 512-bin curves of log(lambda E) (cell axis, then
 *     gene axis);
 *   loss: masked mean squared error against targets resampled the same way;
 *   optimiser: AdamW (0.9, 0.999, eps 1e-8, decoupled weight decay).
 * All arrays are device pointers; spectra are FP64 and descending.
 */
int64_t gmgm_ws_param_count(void);

/* Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) initialisation from a SplitMix64
 * hash of (seed, index).  Asynchronous. */
gmgm_status gmgm_ws_init(gmgm_ctx_t ctx, float* params, uint64_t seed);

/* The 1028 features of an axis pair (E_c: r_c values, E_g: r_g values, both
 * positive; d_c, d_g the axes' dimensions >= 1).  Asynchronous; non-positive
 * E is reported as GMGM_E_DOMAIN by the next synchronising call. */
gmgm_status gmgm_ws_features(gmgm_ctx_t ctx, const double* Ec, int64_t rc, const double* Eg, int64_t rg,
                             double dc, double dg, float* feat);

/* Training targets (1024): resampled log(lambda_c E_c) and log(lambda_g E_g)
 * of a solved problem.  Asynchronous. */
gmgm_status gmgm_ws_targets(gmgm_ctx_t ctx, const double* Ec, const double* lam_c, int64_t rc,
                            const double* Eg, const double* lam_g, int64_t rg, float* target);

/* out (batch x 1024) = network(feats (batch x 1028)); 1 <= batch <= 8192.
 * Asynchronous. */
gmgm_status gmgm_ws_forward(gmgm_ctx_t ctx, const float* params, int32_t batch, const float* feats,
                            float* out);

/* One AdamW step (step >= 1 counts updates) on the masked MSE of a batch.
 * mask: batch x 1024 per-entry weights or NULL (all ones).  adam_m, adam_v:
 * optimiser state (param_count floats each, zero before step 1).  loss_out:
 * host or NULL (then asynchronous; else synchronises): the loss before the
 * update.  grad_out: device or NULL: the gradient (param_count floats). */
gmgm_status gmgm_ws_train_step(gmgm_ctx_t ctx, float* params, float* adam_m, float* adam_v, int64_t step,
                               int32_t batch, const float* feats, const float* target, const float* mask,
                               float lr, float weight_decay, double* loss_out, float* grad_out);

/* Warm-start eigenvalues from one output row: index i of an axis of rank r
 * reads the curve at u_i = (i + 1/2) 512 / r - 1/2 (clamped, linear), and
 * lambda_i = exp(curve(u_i)) / E_i.  Asynchronous. */
gmgm_status gmgm_ws_apply(gmgm_ctx_t ctx, const float* curves, const double* Ec, int64_t rc,
                          const double* Eg, int64_t rg, double* lam_c, double* lam_g);

/*
 * The learned warm start as two calls (the network, features and loss of the
 * gmgm_ws_* calls above; it replaces Algorithm 1's start lambda^0 = 1/E).
 *
 * weights     the network's parameter vector (gmgm_ws_param_count() FP32,
 *             device), e.g. from gmgm_ws_init; updated in place by training.
 * opt_state   device memory of gmgm_warmstart_state_bytes() bytes holding the
 *             AdamW state: an int64 update count at byte 0, the FP32 decoupled
 *             weight decay at byte 8, then the first and second moments
 *             (param_count FP32 each) from byte 256.  gmgm_warmstart_state_init
 *             zeroes it and sets the weight decay.
 */
int64_t gmgm_warmstart_state_bytes(void);

/* Zero the optimiser state and set its weight decay (>= 0).  Asynchronous. */
gmgm_status gmgm_warmstart_state_init(gmgm_ctx_t ctx, void* opt_state, float weight_decay);

/* out (batch x 1024 FP32, device) = network(feats (batch x 1028 FP32,
 * device)); 1 <= batch <= 8192.  Asynchronous. */
gmgm_status gmgm_warmstart_infer(gmgm_ctx_t ctx, const void* weights, int32_t batch, const float* feats,
                                 float* out);

/* One AdamW step (AdamW: 0.9, 0.999, eps 1e-8; the update count in opt_state
 * is incremented on the device and gives the bias corrections) on the masked
 * mean squared error of a batch: feats (batch x 1028), target and mask
 * (batch x 1024 FP32, device; mask NULL = all ones), learning rate lr >= 0.
 * loss_out: host float or NULL; when given, the loss before the update is
 * written and the call synchronises, else it is asynchronous. */
gmgm_status gmgm_warmstart_train_step(gmgm_ctx_t ctx, void* weights, void* opt_state, int32_t batch,
                                      const float* feats, const float* target, const float* mask, float lr,
                                      float* loss_out);

#ifdef __cplusplus
}
#endif

#endif /* GMGM_H */
