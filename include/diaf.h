/*
 * diaf.h -- C ABI of a GPU (MI355X / gfx950) library for preconditioning
 * with direct approximate factoring of the inverse, A^{-1} ~ W V^{-1}
 * (Byckling & Huhtanen, "Preconditioning with direct approximate factoring
 * of the inverse").
 *
 * Method (paper, Sections 1-2): for a sparse nonsingular A and sparse
 * "standard" matrix subspaces (sparsity patterns) for W and V, solve
 * min ||A W - V||_F (eq. 1.2) column by column with the columns of either V
 * or W of fixed (unit) norm.  Column j only touches the columns A(:, J_j)
 * named by the W pattern J_j, so all columns are independent.
 *   - DIAF_UNIT_V (first basic algorithm, Section 2.1): v_j is the unit
 *     vector on the V pattern L_j whose component in range(A(:, J_j)) is
 *     largest (eq. 2.3); w_j solves the least-squares problem (eq. 2.4).
 *   - DIAF_UNIT_W (second basic algorithm, Section 2.2): w_j is the right
 *     singular vector of the smallest singular value of A(:, J_j) with the
 *     rows L_j removed; v_j = (A w_j) restricted to L_j.
 * The V pattern may be fixed, or chosen per column as the optimal one for a
 * seed w (Section 3.1): the diagonal plus the l-1 admissible rows of the
 * triangle with the largest |A w|.  The factors are applied from the right
 * (Section 2.3) inside right-preconditioned BiCGSTAB (Section 5).
 *
 * Conventions
 *   - Every array pointer is a DEVICE pointer unless its name ends in
 *     _host.  Sparse matrices are CSC with int32 colptr[n+1] and int32
 *     rowidx[nnz]; row indices are sorted and unique within each column and
 *     every diagonal entry is present.  Values are double or interleaved
 *     complex double (re, im).
 *   - All work is ordered on the context's HIP stream.  Calls that return
 *     host values (diaf_factor's statistics, diaf_solve) synchronise it.
 *   - Errors are reported by return code only; diaf_last_error() gives a
 *     message for the last failing call on a context.  No call aborts.
 *   - Ownership: the caller owns A, patterns, vectors and every buffer it
 *     passes in.  The library owns the objects it creates (contexts,
 *     factors, models) and their device memory until the matching
 *     *_destroy call.  Views return borrowed pointers valid until then.
 *   - A context must not be used from two host threads at once.
 */
#ifndef DIAF_H
#define DIAF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum diaf_status {
    DIAF_OK = 0,
    DIAF_EINVAL = 1,        /* invalid argument or input (checked before any launch) */
    DIAF_ENOMEM = 2,        /* device allocation failed */
    DIAF_EDEVICE = 3,       /* HIP runtime error */
    DIAF_EUNSUPPORTED = 4,  /* input outside the supported sizes (message says which) */
    DIAF_ESINGULAR = 5,     /* zero or non-finite pivot in V */
    DIAF_ENOCONV = 6,       /* BiCGSTAB did not converge within maxit (the paper's dagger) */
    DIAF_EBREAKDOWN = 7     /* BiCGSTAB breakdown (the paper's double dagger) */
} diaf_status;

typedef enum diaf_dtype { DIAF_F64 = 0, DIAF_C128 = 1 } diaf_dtype;

/* Column norm constraint: unit-norm columns of V (first basic algorithm)
 * or of W (second basic algorithm). */
typedef enum diaf_norm_mode { DIAF_UNIT_V = 0, DIAF_UNIT_W = 1 } diaf_norm_mode;

/* W pattern J (Section 4): pattern(A); pattern(A^2), the truncated Neumann
 * series of Section 4.1 with diagonal V_0, truncation 2 and no dropping;
 * pattern(A) plus the w_topk two-hop rows of largest |A|^2 path weight
 * sum_c |a_ic||a_cj| (dropping by count, Section 4.1); an explicit pattern;
 * or a learned proposal from the A^2 candidates (diaf_model, below). */
typedef enum diaf_w_kind {
    DIAF_W_A = 0, DIAF_W_A2 = 1, DIAF_W_A_1HOP_TOPK = 2, DIAF_W_EXPLICIT = 3, DIAF_W_LEARNED = 4,
    /* Algorithm 2 (Section 4): column j of W has the pattern of A^* v_j for a
     * generic v_j in V_0, i.e. the union of the rows of A at the pattern of
     * column j of V_0; V_0 = diagonal matrices (W = pattern(A^*)), or the
     * Gauss-Seidel structure of Definition 4.1 (diagonal plus the strictly
     * upper / lower part of pattern(A)).  The optional sparsification step
     * of the algorithm is not applied. */
    DIAF_W_ALG2_DIAG = 5, DIAF_W_ALG2_GS_UPPER = 6, DIAF_W_ALG2_GS_LOWER = 7,
    /* Algorithm 1 (Section 4), sparsified powers with V_0 the diagonal
     * matrices, real A only (DIAF_EUNSUPPORTED for DIAF_C128): parameters in
     * diaf_spec.sparsify / diaf_pattern_build_sparsified. */
    DIAF_W_SPARSIFIED = 8
} diaf_w_kind;

/* Parameters of the sparsified powers W pattern (Section 4, Algorithm 1),
 * real or complex A.  The splitting A = V_0 (I - S) with V_0 = P_{V_0} A
 * gives S = V_0^{-1}(A - P_{V_0} A): for V_0 the diagonal matrices
 * (v0_nblocks = 0), S(i, c) = a_ic / a_ii off the diagonal; for V_0 the
 * block diagonal matrices with the given blocks (Section 4's other
 * inexpensive choice), V_0 is A's block diagonal part, each block is
 * factored with partial pivoting, and column c of S is the block solve of
 * A(:, c) outside c's block, every row of every block it reaches being an
 * entry.  Each column of S is first sparsified by (tau_i, p_i); then, for
 * every column j, t = e_j is multiplied by S k times, each product
 * sparsified by (tau_l, p_l) with its entry in row j never dropped, and the
 * pattern of w_j is the union of e_j and every kept t, less the rows of
 * j's block other than j (the algorithm's final removal of V_0 minus the
 * identity).  Dropping by tolerance keeps the entries with |v|^2 >= tau^2
 * max |v|^2 over the vector; dropping by count then keeps the p largest
 * (equal magnitudes: the lower rows); a zero parameter disables its rule.
 * Products are summed in ascending source row with round-to-nearest
 * operations (complex: (ar br - ai bi, ar bi + ai br), and a / d as
 * a conj(d) / |d|^2), so with the diagonal V_0 the pattern is reproducible
 * bit for bit; with blocks the LU solves round differently from other LU
 * codes, and only decisions within rounding of a dropping boundary can
 * differ.  k in 1..8; p_i, p_l in 0..2^20; tau_i, tau_l finite and >= 0;
 * v0_blocks given exactly when v0_nblocks > 0, its starts running from 0 to
 * n and increasing (else DIAF_EINVAL); a zero diagonal entry or a singular
 * diagonal block is DIAF_EINVAL; a block of more than 64 rows, a column of
 * A or of S before dropping with more than 1024 entries, a power vector of
 * more than 2048 rows (complex 1024) or a pattern of more than 4096 rows
 * (complex 2048) is DIAF_EUNSUPPORTED. */
typedef struct diaf_sparsify {
    int32_t k;          /* truncation of the series I + S + ... + S^k */
    int32_t p_i;        /* count limit on the columns of S */
    int32_t p_l;        /* count limit on every power vector t */
    int32_t v0_nblocks; /* 0: V_0 diagonal; else the number of diagonal blocks of V_0 */
    double tau_i;       /* relative tolerance on the columns of S */
    double tau_l;       /* relative tolerance on every power vector t */
    const int32_t* v0_blocks; /* device array of v0_nblocks + 1 block starts
                                 0 = s_0 < ... < s_m = n (blocks of at most
                                 64 rows), or NULL */
} diaf_sparsify;

/* V pattern L: explicit; diagonal; Gauss-Seidel structure (Definition 4.1:
 * diagonal plus the strictly upper / lower part of pattern(A)); the optimal
 * choice for the seed w (Section 3.1): the diagonal plus the v_count-1 rows
 * of the upper / lower triangle of the shadow R_j with the largest |A w0|,
 * w0 being the solution for V_0 = diagonals (TOPK); or Section 3.1's own
 * suboptimal rule for DIAF_UNIT_V: the diagonal plus the v_count-1 rows of
 * the triangle whose columns of Q_j^* (A_j = Q_j R_j) have the largest norm,
 * i.e. the largest leverage b_i (A_j^* A_j)^{-1} b_i^* (LEV; DIAF_EINVAL with
 * DIAF_UNIT_W).  Ties within 1e-10 relative go to the lower row. */
typedef enum diaf_v_kind {
    DIAF_V_EXPLICIT = 0, DIAF_V_DIAG = 1, DIAF_V_GS_UPPER = 2, DIAF_V_GS_LOWER = 3,
    DIAF_V_TOPK_UPPER = 4, DIAF_V_TOPK_LOWER = 5, DIAF_V_LEV_UPPER = 6, DIAF_V_LEV_LOWER = 7,
    /* Block diagonal V (Section 5: V the block diagonal matrices of the
     * splitting A = L + D + U; consecutive blocks given by diaf_spec.v_blocks,
     * at most 64 rows each, else DIAF_EUNSUPPORTED): the pattern of D, i.e.
     * the rows of A(:, j) inside j's block (BLOCK), or the diagonal plus the
     * v_count-1 other rows of j's block with the largest |A w0|, w0 as for
     * TOPK (TOPK_BLOCK).  V^{-1} is applied through an LU with partial
     * pivoting of each block, computed on the first apply or solve; a
     * singular block makes them return DIAF_ESINGULAR. */
    DIAF_V_BLOCK = 8, DIAF_V_TOPK_BLOCK = 9
} diaf_v_kind;

/* Per-column flag bits (diaf_view.flags). */
#define DIAF_FLAG_RANK_DEFICIENT 1u /* B = A(R_j, J_j) numerically rank deficient: unit-norm v, the
                                       Gram pivots |R_aa|^2 of B = QR reach 1e-14 times the largest
                                       squared column norm (or |J_j| > |R_j|); unit-norm w, B without
                                       the rows L_j has sigma_min^2 <= 1e-14 times its squared
                                       Frobenius norm (or fewer rows than columns) */
#define DIAF_FLAG_GAP_DEGENERATE 2u /* extreme singular values not separated (rel. gap < 1e-6) */
#define DIAF_FLAG_SMALL_DIAG 4u     /* |v_jj| < 1e-2 ||v_j|| */
#define DIAF_FLAG_FELL_BACK 8u      /* learned pattern rejected by the residual gate */
#define DIAF_FLAG_TIE_EDGE 16u      /* a top-k score at the edge of the 1e-10 tie band */
#define DIAF_FLAG_STABILIZED 32u    /* v_j computed under the constraint v_jj = stab_r (Section 3.2) */
#define DIAF_FLAG_NO_DIAG_ROW 64u   /* row j not in the shadow of J_j: column left zero */
#define DIAF_FLAG_NULL_CHOICE 128u  /* unit-norm w: the block without the rows L_j has a null space
                                       of dimension >= 2; w is its unit vector with the largest
                                       |(A w)_j| (Section 2.2 with Theorem 2.1's v_jj != 0) */

typedef struct diaf_csc {
    int64_t n, nnz;
    const int32_t* colptr;
    const int32_t* rowidx;
    const void* val;   /* nnz doubles (DIAF_F64) or nnz (re, im) pairs (DIAF_C128) */
    int32_t dtype;     /* diaf_dtype */
} diaf_csc;

typedef struct diaf_pattern {
    int64_t n, nnz;
    const int32_t* colptr;
    const int32_t* rowidx;
} diaf_pattern;

struct diaf_ctx;
struct diaf_factors;
struct diaf_model;

typedef struct diaf_spec {
    int32_t w_kind;                  /* diaf_w_kind */
    int32_t w_topk;                  /* DIAF_W_A_1HOP_TOPK: extra rows per column */
    const diaf_pattern* w_explicit;  /* DIAF_W_EXPLICIT: must contain every diagonal */
    struct diaf_model* model;        /* DIAF_W_LEARNED */
    double gate_tau;                 /* DIAF_W_LEARNED: refactor with pattern(A^2) when
                                        r_j / s_j > gate_tau (s_j = 1 for DIAF_UNIT_V,
                                        ||A(:,J_j)||_F for DIAF_UNIT_W) */
    int32_t v_kind;                  /* diaf_v_kind */
    int32_t v_count;                 /* DIAF_V_TOPK_*: l, counting the diagonal */
    const diaf_pattern* v_explicit;  /* DIAF_V_EXPLICIT (rows outside the shadow get 0) */
    int32_t gram_fp32;               /* 1: Gram matrix accumulated in FP32 products (variant) */
    double gate_dom;                 /* DIAF_W_LEARNED: also refactor with pattern(A^2) when
                                        |v_jj| < gate_dom * sum_{i != j} |v_ij| for the
                                        proposal's V column: chains of such columns make the
                                        triangular solve with V grow exponentially (0 = off) */
    double stab_r;                   /* Section 3.2, DIAF_UNIT_V with a triangular V rule
                                        (DIAG, GS_*, TOPK_*): a column whose |v_jj| falls
                                        below stab_tol * ||v_j|| is recomputed with
                                        v_jj = stab_r, the other rows of L_j carrying the
                                        unit vector of Section 3.2, w_j the least-squares
                                        solution for that v_j; flag DIAF_FLAG_STABILIZED
                                        (0 = off; the paper's experiment uses 2) */
    double stab_tol;                 /* trigger of stab_r (the paper's experiment: 1e-2) */
    diaf_sparsify sparsify;          /* DIAF_W_SPARSIFIED */
    const int32_t* v_blocks;         /* DIAF_V_BLOCK / DIAF_V_TOPK_BLOCK: device array of
                                        v_nblocks + 1 block starts, 0 = s_0 < ... = n */
    int32_t v_nblocks;
    int32_t left;                    /* 1: the left variant (Section 2.3's remarks on left and
                                        right approximate inverses): W A ~ V, found by the
                                        columnwise method on A^* (every pattern and rule above
                                        then applies to A^*, W^*, V^*; a lower rule gives an
                                        upper V), M = V^{-1} W; diaf_apply computes V^{-1} W x
                                        and diaf_solve runs BiCGSTAB on M A x = M b, stopped on
                                        the preconditioned residual (relres), relres_true still
                                        ||b - A x|| / ||b||.  0: right (eq. 2.1) */
} diaf_spec;

/* Borrowed device views of a factorization.  W has the pattern J (Wcp/Wri)
 * and values Wval; V is CSC with sorted rows.  r[j] = ||A w_j - v_j||_2,
 * flags[j] as above, lcount[j] = |L_j|.  vtri = 1 upper, -1 lower,
 * 0 diagonal, 3 block diagonal (DIAF_V_BLOCK, DIAF_V_TOPK_BLOCK), 2 none of
 * these (an explicit V pattern; diaf_apply and diaf_solve then return
 * DIAF_EUNSUPPORTED). */
typedef struct diaf_view {
    int64_t n, nnz_w, nnz_v;
    int32_t dtype, vtri;
    const int32_t* Wcp;
    const int32_t* Wri;
    const void* Wval;
    const int32_t* Vcp;
    const int32_t* Vri;
    const void* Vval;
    const double* r;
    const uint32_t* flags;
    const int32_t* lcount;
} diaf_view;

/* Host statistics gathered by diaf_factor. */
typedef struct diaf_stats {
    int64_t n, nnz_w, nnz_v;
    int32_t kmax, mmax;              /* largest |J_j| and shadow size bound */
    int32_t nbuckets;                /* size classes launched */
    int32_t count_rank_deficient, count_gap_degenerate, count_small_diag, count_tie_edge,
        count_fell_back, count_no_diag;
    int32_t v_levels;                /* dependency depth of the V solve: 1 for a
                                        (block) diagonal V after the first apply
                                        or solve, for a triangular V after
                                        diaf_factors_levels (0 before) */
    int32_t count_zero_pivot;        /* zero / non-finite diagonal entries of V (idem) */
    int32_t factor_launches;         /* factor kernel launches (one per size class) */
    int32_t count_deferred;          /* columns the small-column kernel handed to the
                                        generic one */
    double nrm;                      /* ||A W - V||_F = sqrt(sum r_j^2) */
    double ms_pattern, ms_factor, ms_assemble;  /* device time of the phases */
    double ms_factor_kernels;        /* device time of the factor kernels alone */
    int32_t count_stabilized;        /* columns computed under the Section 3.2 constraint */
    int32_t count_null_choice;       /* columns with DIAF_FLAG_NULL_CHOICE */
    /* Device time and columns per factor kernel, summed over the factoring
     * passes of these factors (the fallback pass of a learned pattern
     * included): the one-wave kernel (the columns it finished, not those it
     * handed on), and the generic kernel per size class (the capacities of
     * class c are class_kcap[c] and class_tcap[c] below; with the default
     * table, classes 0..6 hold |J_j| <= 16/32/64/64/128/256/256 and gathered
     * entries <= 128/256/512/1024/2048/4096/8192). */
    double ms_small_kernel;
    double ms_generic_class[8];
    int32_t cols_small;
    int32_t launches_small;
    int32_t cols_generic_class[8];
    int32_t launches_generic_class[8];
    /* Theoretical occupancy of those launches, in waves per SIMD (the
     * runtime's occupancy calculator with the kernels' register and LDS
     * use; 0 where nothing ran). */
    double occ_small;
    double occ_generic_class[8];
    /* The mid-size one-wave kernel (unit-norm v, shadows beyond 64 rows):
     * device time, columns it finished, launches and occupancy. */
    double ms_mid_kernel;
    int32_t cols_mid;
    int32_t launches_mid;
    double occ_mid;
    /* Capacities (|J_j|, gathered entries) of the size classes of the last
     * factoring pass (the context option "class_table"); 0 past the last. */
    int32_t class_kcap[8];
    int32_t class_tcap[8];
} diaf_stats;

typedef struct diaf_solve_info {
    int32_t iters;       /* BiCGSTAB iterations (half steps rounded up) */
    int32_t flag;        /* 0 converged, 1 maxit, 2 breakdown, 3 singular V */
    double relres;       /* recurrence residual / ||b|| at exit */
    double relres_true;  /* ||b - A x|| / ||b|| recomputed at exit */
    double ms;           /* wall time of the solve */
} diaf_solve_info;

/* ---- context ---------------------------------------------------------- */

/* Create a context on HIP device `device` that orders all work on
 * `hip_stream` (a hipStream_t; NULL = the null stream).
 *
 * Device memory: the library keeps the blocks it frees (up to 32 GiB per
 * device, shared by all contexts on that device) and reuses them in later
 * calls instead of calling hipMalloc and hipFree each time; it releases them
 * when hipMalloc runs out of memory.  Freeing a block waits for the device
 * to be idle, as hipFree does. */
diaf_status diaf_ctx_create(struct diaf_ctx** ctx, int device, void* hip_stream);
/* Waits for the device, releases the device memory the library keeps for
 * this context's device, and frees the context. */
void diaf_ctx_destroy(struct diaf_ctx* ctx);
const char* diaf_last_error(const struct diaf_ctx* ctx);

/* Copy `bytes` between two buffers of any kind (device or host, the
 * runtime tells which) in the context's stream order, then synchronise the
 * stream: a helper for bindings that marshal host arrays into the device
 * buffers the other calls take.  Errors: DIAF_EINVAL (NULL context, or a
 * NULL buffer with bytes > 0), DIAF_EDEVICE. */
diaf_status diaf_copy(struct diaf_ctx* ctx, void* dst, const void* src, size_t bytes);
/* Tunables of the context (not of the method: results are identical for
 * every setting of the launch shapes; "generic_only" and "mid" route columns
 * to another kernel of the same method, whose results agree to rounding).
 * Keys:
 *   "generic_only"       1: every column goes to the generic factor kernel
 *   "mid"                0: no mid-size one-wave kernel (unit-norm v columns
 *                        with shadows beyond 64 rows go to the generic kernel)
 *   "class_table"        size classes of the factor launches (0 default, 0..3;
 *                        every table sends the same columns to each kernel)
 *   "factor_graph"       1 (default): diaf_refactor replays the recorded factor
 *                        launches (unit-norm v) as one captured graph
 *   "small_grid"         workgroups of the one-wave factor kernel (0 = 4096)
 *   "generic_nt"         threads per column of the generic kernel (0 auto, 64,
 *                        128, 256, 512)
 *   "solve_batch"        BiCGSTAB iterations between host polls (>= 1)
 *   "graph"              1: replay each batch from one captured hipGraph
 *   "trsv_backoff"       0..256: a triangular-solve wave that made no progress
 *                        sleeps 64, 128, 256, ... cycles, up to 64 x the value,
 *                        before polling again (0: never; default 1)
 *   "trsv_waves"         waves per workgroup of the triangular solve (1, 2, 4,
 *                        8, 16; default 8): the workgroup owns 64 x waves
 *                        consecutive rows, one per lane, sharing their values
 *                        through LDS; up to 8 waves each row keeps 16 (complex
 *                        12) off-diagonal entries in LDS, at 16 waves 12 (6)
 *   "gate_small_diag"    1: the learned path also rejects proposals whose V
 *                        diagonal entry is flagged negligible
 * DIAF_EINVAL for an unknown key or value.  get_option reads a value. */
diaf_status diaf_ctx_set_option(struct diaf_ctx* ctx, const char* key, int64_t value);
diaf_status diaf_ctx_get_option(const struct diaf_ctx* ctx, const char* key, int64_t* value);

/* Autotuner for the batched factoring and the solve: times the candidate
 * launch shapes on this problem (A, spec, mode, as for diaf_factor) and keeps
 * the fastest in ctx: "small_grid" (1024 ... 16384), "class_table" and
 * "generic_nt" (when generic buckets occur), "trsv_waves", then "graph",
 * "solve_batch" and "trsv_backoff" by the wall time per iteration of
 * 32-iteration solves with b = ones.  Runs a few dozen factorizations and
 * solves; blocks until done.  Leaves the method's results unchanged. */
diaf_status diaf_autotune(struct diaf_ctx* ctx, const diaf_csc* A, const diaf_spec* spec,
                          int32_t mode);
/* diaf_autotune with a persistent store: `path` names a JSON file (one object
 * per line) keyed by the device architecture (gcnArchName) and the problem's
 * shape (mode, dtype, n, nnz, W and V kinds and counts, left, FP32 Gram).  A
 * stored entry for this key is applied to ctx without timing anything
 * (*from_cache = 1); otherwise diaf_autotune runs and its choice is added to
 * the file (*from_cache = 0), written to path + ".tmp" and renamed.  A missing
 * file counts as empty.  Errors: DIAF_EINVAL for a file that is not in this
 * format (it is left untouched) or cannot be written, and those of
 * diaf_autotune.  Concurrent writers of one file: the last rename wins. */
diaf_status diaf_autotune_cached(struct diaf_ctx* ctx, const diaf_csc* A, const diaf_spec* spec,
                                 int32_t mode, const char* path, int32_t* from_cache);

/* ---- patterns (Section 4) ------------------------------------------------ */

/* W pattern of kind w_kind (A, A2, A_1HOP_TOPK, ALG2_*) for A, two-phase: with rowidx_out == NULL,
 * writes colptr_out[n+1] (device) and the total to *nnz_host; then call
 * again with rowidx_out of *nnz_host entries and the same colptr_out.
 * DIAF_EUNSUPPORTED when a column has more candidates than a workgroup's
 * LDS holds: for A2, 8192 (the sum of |A(:, c)| over the rows c of
 * A(:, j)); for A_1HOP_TOPK, 4095 - w_topk two-hop candidates, w_topk <= 256. */
diaf_status diaf_pattern_build(struct diaf_ctx* ctx, const diaf_csc* A, int32_t w_kind,
                               int32_t w_topk, int32_t* colptr_out, int32_t* rowidx_out,
                               int64_t* nnz_host);

/* The sparsified powers W pattern (Section 4, Algorithm 1; parameters and
 * errors as for diaf_sparsify) for real A, two-phase like
 * diaf_pattern_build: colptr_out[n+1] (device) and *nnz_host first, then
 * rowidx_out (device, *nnz_host entries, ascending rows per column). */
diaf_status diaf_pattern_build_sparsified(struct diaf_ctx* ctx, const diaf_csc* A,
                                          const diaf_sparsify* prm, int32_t* colptr_out,
                                          int32_t* rowidx_out, int64_t* nnz_host);

/* ---- factoring (Sections 2-3) -------------------------------------------- */

/* Factor A W ~ V with the given patterns and norm mode.  On success *out
 * owns W, V, the residuals and flags.  DIAF_EINVAL for malformed input
 * (unsorted or duplicate rows, missing diagonal, non-finite values, bad
 * spec); DIAF_EUNSUPPORTED for columns beyond the kernel size limits
 * (|J_j| <= 256, gathered entries <= 8192). */
diaf_status diaf_factor(struct diaf_ctx* ctx, const diaf_csc* A, const diaf_spec* spec,
                        int32_t mode, struct diaf_factors** out);
diaf_status diaf_factors_view(const struct diaf_factors* F, diaf_view* out_host);
diaf_status diaf_factors_stats(const struct diaf_factors* F, diaf_stats* out_host);
/* Dependency depth of the V solve, a diagnostic of the sync-free
 * triangular solve (the method only asks that V be easily invertible, as a
 * triangular matrix is, Section 1): the number of steps of the longest
 * chain of rows of a triangular V that each wait on the previous one, 1 for
 * a diagonal or block diagonal V.  Builds the apply
 * copies when no apply or solve has yet, then walks the rows of V on ctx's
 * stream and waits for the result.  The value is kept in the statistics
 * (v_levels, 0 for a triangular V until this call).  Errors: DIAF_EINVAL
 * (NULL argument), DIAF_EUNSUPPORTED (V neither triangular nor (block)
 * diagonal), DIAF_EDEVICE. */
diaf_status diaf_factors_levels(struct diaf_ctx* ctx, const struct diaf_factors* F,
                                int32_t* levels);
void diaf_factors_destroy(struct diaf_factors* F);

/* ---- apply and solve (eq. 2.1, Section 5) -------------------------------- */

/* Refactor F in place for new values of the matrix it was built from: A
 * must be the same descriptor contents as at diaf_factor (the same colptr,
 * rowidx and val buffers, n and nnz), with new values written into val and
 * the pattern unchanged (checked against a 64-bit fingerprint taken at
 * factor time).  The W pattern and V's capacity are kept; the columns are
 * factored again with F's spec and mode (the V pattern rule runs again, as
 * Section 3.1's selection depends on the values), V is assembled and the
 * statistics retaken; the apply structures are rebuilt on the next apply.
 * The first refactor runs the factor launches eagerly and records them;
 * for DIAF_UNIT_V later calls replay them as one captured hipGraph (context
 * option "factor_graph", default 1); unit-norm w, whose hand-over of
 * rank-deficient columns depends on the values, always runs eagerly.
 * Results are those of diaf_factor on the new values.  Errors: DIAF_EINVAL
 * (other buffers or sizes, a changed pattern, factors of another context,
 * or a replay whose hand-over counts differ from the recorded pass: factor
 * afresh), DIAF_EUNSUPPORTED (the left variant, or a W pattern that depends
 * on the values: 1-hop, sparsified powers, learned), DIAF_EDEVICE.  For
 * time stepping with a fixed sparsity pattern (Section 5's setting of
 * repeated solves). */
diaf_status diaf_refactor(struct diaf_ctx* ctx, const diaf_csc* A, struct diaf_factors* F);

/* y = W V^{-1} x for triangular, diagonal or block diagonal V (n entries
 * each); y = V^{-1} W x for factors of the left variant (diaf_spec.left).
 * DIAF_ESINGULAR when V has a zero or non-finite pivot. */
diaf_status diaf_apply(struct diaf_ctx* ctx, const struct diaf_factors* F, const void* x,
                       void* y);

/* diaf_apply for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same kernels and the same result, bit for bit, with the intermediate
 * vector and the triangular solve's control words in a fixed scratch array
 * of 16 MiB that each device holds from diaf_ctx_create until the process
 * ends; it calls no hipMalloc or hipFree.  x, y: n entries each, caller
 * owned.  Limits and errors: n * (8 or 16 bytes) must fit in 16 MiB - 256 B
 * (n <= 2 097 120 real, 1 048 560 complex), else DIAF_EINVAL; the factors
 * must have been prepared by one diaf_apply or diaf_solve (which build
 * their row-oriented copies), else DIAF_EINVAL; DIAF_ESINGULAR as for
 * diaf_apply.  All calls on one device share its scratch array: calls that
 * overlap in time on one device (other streams, other threads) race, and
 * must be ordered by the caller. */
diaf_status diaf_apply_noalloc(struct diaf_ctx* ctx, const struct diaf_factors* F,
                               const void* x, void* y);

/* Right-preconditioned BiCGSTAB on A M u = b, x = M u, M = W V^{-1}
 * (F == NULL: M = I), x0 = 0, stop when ||r|| <= rtol ||b||; for factors of
 * the left variant, BiCGSTAB on M A x = M b, M = V^{-1} W, stop when the
 * preconditioned residual ||M (b - A x)|| <= rtol ||M b||.  Returns
 * DIAF_OK, DIAF_ENOCONV, DIAF_EBREAKDOWN or DIAF_ESINGULAR (V has a zero
 * pivot: x = 0, info flag 3) with *info_host filled. */
diaf_status diaf_solve(struct diaf_ctx* ctx, const diaf_csc* A, const struct diaf_factors* F,
                       const void* b, void* x, double rtol, int32_t maxit,
                       diaf_solve_info* info_host);

/* ---- learned W-pattern proposer ------------------------------------------ */
/*
 * A multilayer perceptron 16 -> 64 -> 64 -> 1 (ReLU, FP32) scores each
 * candidate i of column j's A^2 pattern from 16 column-local features; the
 * proposal is J_j = {j} U {i : sigmoid(score) >= 0.5}.  Parameters are one
 * float array of DIAF_MLP_NPARAM entries: W1[64][16], b1[64], W2[64][64],
 * b2[64], w3[64], b3 (row-major, y = W x + b).
 */
#define DIAF_MLP_NFEAT 16
#define DIAF_MLP_HIDDEN 64
#define DIAF_MLP_NPARAM (64 * 16 + 64 + 64 * 64 + 64 + 64 + 1)

/* Create a model holding a copy of params_host (DIAF_MLP_NPARAM floats). */
diaf_status diaf_model_create(struct diaf_ctx* ctx, const float* params_host,
                              struct diaf_model** out);
diaf_status diaf_model_get_params(struct diaf_ctx* ctx, const struct diaf_model* m,
                                  float* params_host);
void diaf_model_destroy(struct diaf_model* m);

/* Features of every (column j, candidate i) pair of the candidate pattern
 * C (CSC; normally pattern(A^2)), written as feat[nnz(C)][16] floats. */
diaf_status diaf_features(struct diaf_ctx* ctx, const diaf_csc* A, const diaf_pattern* C,
                          float* feat);

/* Labels of the candidates from a plain factorization F whose W pattern is
 * C: label = 1 when |w_j(i)| ||A(:,i)|| >= tau * max over the column, and
 * always for i = j (dropping by tolerance, Section 4.1). */
diaf_status diaf_labels(struct diaf_ctx* ctx, const diaf_csc* A, const struct diaf_factors* F,
                        double tau, float* labels);

/* scores[p] = MLP(feat[p]) for p < npairs. */
diaf_status diaf_mlp_forward(struct diaf_ctx* ctx, const struct diaf_model* m, const float* feat,
                             int64_t npairs, float* scores);

/* Mean binary cross-entropy loss of the logits against labels (0/1 floats)
 * and its gradient with respect to the parameters (grad: DIAF_MLP_NPARAM
 * floats, device; may be NULL).  *loss_host receives the loss. */
diaf_status diaf_mlp_loss_grad(struct diaf_ctx* ctx, const struct diaf_model* m,
                               const float* feat, const float* labels, int64_t npairs,
                               float* grad, double* loss_host);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) on the mean BCE loss of
 * the given pairs.  The model keeps its moment estimates and step count. */
diaf_status diaf_mlp_train_step(struct diaf_ctx* ctx, struct diaf_model* m, const float* feat,
                                const float* labels, int64_t npairs, float lr,
                                double* loss_host);

#ifdef __cplusplus
}
#endif

#endif /* DIAF_H */
