// Launchers exported by the kernel files to the API layer.
#pragma once

#include "dcommon.h"

namespace diaf {

// ---- patterns (pattern.hip) ----
// Union patterns: column j is the union of the inner lists (Icp/Iri) named
// by the outer list of column j (Ocp/Ori); pattern(A^2) takes the columns of
// A for both.  cnt[j] = the total length of those inner lists, *maxcnt_dev
// the maximum.
Err launch_cand_count(int n, const int32_t* Ocp, const int32_t* Ori, const int32_t* Icp,
                      int32_t* cnt, int32_t* maxcnt_dev, hipStream_t st);
// Symbolic union pattern: count (Jri == nullptr: writes cnt[j]) or fill.
Err launch_pattern_a2(int n, const int32_t* Ocp, const int32_t* Ori, const int32_t* Icp,
                      const int32_t* Iri, int maxcand, int32_t* cnt, const int32_t* Jcp,
                      int32_t* Jri, hipStream_t st);
// Pattern of V_0 for Algorithm 2 (v0 = 0 diagonal, 1 / 2 Gauss-Seidel upper /
// lower): count (Vri == nullptr: writes cnt[j]) or fill.
Err launch_v0_pattern(int n, const int32_t* Acp, const int32_t* Ari, int v0, int32_t* cnt,
                      const int32_t* Vcp, int32_t* Vri, hipStream_t st);
// pattern(A) plus the ptop two-hop rows of largest |A|^2 path weight, for
// the columns cols: cnt[j] rows, ascending, into column j's slot of Jtmp at
// Acp[j] + j ptop (capacity |A(:, j)| + ptop); launch_compact_slots then
// packs the slots at Jcp.
template <class T>
Err launch_pattern_1hop(int n, const int32_t* Acp, const int32_t* Ari, const T* Aval, int ptop,
                        int cand_max, const int32_t* cols, int ncols, int32_t* cnt,
                        int32_t* Jtmp, hipStream_t st);
Err launch_compact_slots(int n, const int32_t* Acp, int ptop, const int32_t* cnt,
                         const int32_t* Jtmp, const int32_t* Jcp, int32_t* Jri, hipStream_t st);
// Sparsified powers (Algorithm 1, real or complex A).  Diagonal V_0: d =
// diag(A) (bit 0 of *bad on a zero); S = D^{-1}(A - D) sparsified by (tau,
// p) per column in A's column layout with scnt[c] entries.  Block diagonal
// V_0 (rb: per row its block's rows [rb[2i], rb[2i+1]); bid: its block):
// D = A's block diagonal part in CSC (count pass, then fill), its blocks
// factored by launch_block_lu, and S built by block solves in its own
// layout Scp (count pass, then fill).  Bit 1 of *bad: a column of A, or of
// S before dropping, longer than 1024.  The level expansion for cols (null:
// all n columns), count (Jri null: cnt[j]) or fill, with the rows of j's
// block other than j removed (rb null: no removal), columns outgrowing the
// LDS tables appended to over.
constexpr int SP_TC_SMALL = 256, SP_SC_SMALL = 512;    // power vector / pattern rows
template <class T>
struct SpCaps {  // the larger LDS tables (complex values take twice the room)
    static constexpr int TL = num<T>::is_complex ? 1024 : 2048;
    static constexpr int SL = num<T>::is_complex ? 2048 : 4096;
};
template <class T>
Err launch_sp_diag(int n, const int32_t* Acp, const int32_t* Ari, const T* Aval, T* d,
                   int32_t* bad, hipStream_t st);
template <class T>
Err launch_sp_build_s(int n, const int32_t* Acp, const int32_t* Ari, const T* Aval, const T* d,
                      double tau, int p, int32_t* Sri, T* Sval, int32_t* scnt, int32_t* bad,
                      hipStream_t st);
template <class T>
Err launch_sp_block_d(int n, const int32_t* Acp, const int32_t* Ari, const T* Aval,
                      const int32_t* rb, int32_t* cnt, const int32_t* Dcp, int32_t* Dri, T* Dval,
                      hipStream_t st);
template <class T>
Err launch_sp_build_s_block(int n, const int32_t* Acp, const int32_t* Ari, const T* Aval,
                            const int32_t* rb, const int32_t* bid, const int32_t* bstart,
                            const int64_t* boff, const T* LU, const int32_t* perm, double tau,
                            int p, int32_t* scnt, const int32_t* Scp, int32_t* Sri, T* Sval,
                            int32_t* bad, hipStream_t st);
template <class T>
Err launch_sp_expand(int n, const int32_t* Scp, const int32_t* Sri, const T* Sval,
                     const int32_t* scnt, int k, double tau, int p, const int32_t* rb,
                     const int32_t* cols, int ncols, int large, int32_t* cnt, const int32_t* Jcp,
                     int32_t* Jri, int32_t* over, int32_t* nover, hipStream_t st);
// Per-column sizes for bucketing: k[j] = |J_j|, t[j] = sum nnz(A(:, J_j)).
Err launch_column_sizes(int n, const int32_t* Acp, const int32_t* Jcp, const int32_t* Jri,
                        int32_t* kout, int32_t* tout, hipStream_t st);
// Size classes of the factor launches (capacity in |J_j| and in gathered
// entries), smallest first.
struct ColumnClasses {
    static constexpr int kMax = 8;
    int ncls;
    int kcap[kMax];
    int tcap[kMax];
};
// The m columns sel[0..m) (0..m-1 when sel is null) stably sorted by class
// into sorted[0..m); counts[0..ncls] per class (ncls: fits none); maxes[0..1]
// the largest k and t over all n columns (null: not taken).
Err launch_classify_columns(int n, int m, const int32_t* sel, const int32_t* kk, const int32_t* tt,
                            const ColumnClasses& cc, int32_t* sorted, int32_t* counts,
                            int32_t* maxes, hipStream_t st);
// Ascending sort of m column indices below n.
Err sort_columns(int n, int m, const int32_t* in, int32_t* out, hipStream_t st);

// ---- factoring (factor_generic.hip, factor_small.hip) ----
// gws: global workspace of generic_global_bytes(...) bytes (may be null when
// that is 0); nslots = number of blocks sharing it.
// Launch shapes chosen by the autotuner (0 = built-in choice).
struct FactorTune {
    int small_grid = 0;  // workgroups of the one-wave kernel (persistent over columns)
    int generic_nt = 0;  // threads per column of the generic kernel (64, 128, 256 or 512)
};
template <class T>
Err launch_factor_generic(const FactorArgs<T>& A, int kcap, int tcap, int lcap, void* gws,
                          int nslots, FactorTune tune, hipStream_t st);
template <class T>
size_t generic_global_bytes(int kcap, int tcap, int lcap, int mode, int nslots);
// One-wave kernel for unit-norm v and |J_j| <= 32, shadow <= 64, gathered
// entries <= 256, |L_j| <= 8; other columns are appended to deferred.
template <class T>
Err launch_factor_small(const FactorArgs<T>& A, int* deferred, int* ndeferred, FactorTune tune,
                        hipStream_t st);
// One-wave kernel for unit-norm v with |J_j| <= 64 and up to 1024 gathered
// entries (complex: 32 and 256) for shadows beyond 64 rows; columns with more
// than 256 rows holding two or more entries, or |L_j| > 8, are appended to
// deferred.  kcap, tcap: the size class of the launch.
template <class T>
bool mid_supports(int kcap, int tcap);
// The mid-size kernel's own size classes (capacities in |J_j| and gathered
// entries, at most ColumnClasses::kMax); returns their number.
template <class T>
int mid_classes(int* kcap, int* tcap);
template <class T>
Err launch_factor_mid(const FactorArgs<T>& A, int kcap, int tcap, int* deferred, int* ndeferred,
                      FactorTune tune, hipStream_t st);
template <class T>
double mid_occupancy(int kcap, int tcap);
// Theoretical waves per SIMD of the factor kernels (the runtime's occupancy
// calculator): the one-wave kernel, and the generic kernel for a size class
// as launch_factor_generic would place it.
template <class T>
double small_occupancy(int mode);
template <class T>
double generic_occupancy(int kcap, int tcap, int lcap, int mode, FactorTune tune);

// ---- assembly and sparse utilities (sparse.hip) ----
// Temporary device block for work queued on st, released with afree(p, st)
// after the last launch that uses it (no synchronization either way: the
// block is reused only once a later synchronization of st has passed).
Err amalloc(void** p, size_t bytes, hipStream_t st);
void afree(void* p, hipStream_t st);
// Exclusive scan of n ints into out[n+1] (out[n] = total); temp via hipcub.
Err exclusive_scan_i32(const int32_t* in, int32_t* out, int n, hipStream_t st);
template <class T>
Err launch_compact_v(int n, int lmax, const int32_t* lcount, const int32_t* Vcp,
                     const int32_t* Vrows, const T* Vvals, int32_t* Vri, T* Vval, hipStream_t st);
// v <- conj(v) (a no-op for double).
template <class T>
Err launch_conj(int64_t n, T* v, hipStream_t st);
// CSC -> CSR transpose with rows sorted by column (deterministic).
template <class T>
Err csc_to_csr(int n, int64_t nnz, const int32_t* cp, const int32_t* ri, const T* val,
               int32_t* rp, int32_t* ci, T* cval, hipStream_t st);
// Validation of a CSC input: sorted unique in-range rows, diagonal present,
// finite values.  *bad_dev receives a nonzero code for the first problem.
template <class T>
Err launch_validate_csc(int n, const int32_t* cp, const int32_t* ri, const T* val,
                        int32_t* bad_dev, hipStream_t st);
Err launch_validate_pattern(int n, const int32_t* cp, const int32_t* ri, int need_diag,
                            int32_t* bad_dev, hipStream_t st);
template <class T>
Err launch_diag_check(int n, const int32_t* rp, const int32_t* ci, const T* val, int32_t* bad_dev,
                      hipStream_t st);
// 64-bit fingerprint of the pattern (colptr, rowidx) into *out.
Err launch_pattern_hash(int n, int64_t nnz, const int32_t* cp, const int32_t* ri,
                        unsigned long long* out, hipStream_t st);
template <class T>
Err launch_flag_stats(int n, const uint32_t* flags, const double* r, int32_t* counts_dev,
                      double* nrm2_dev, hipStream_t st);
// |v_jj| / sum_{i != j} |v_ij| per column of the padded V layout.
template <class T>
Err launch_col_dominance(int n, int lmax, const int32_t* Vrows, const T* Vvals,
                         const int32_t* lcount, double* dom, hipStream_t st);

// ---- block diagonal V (blockv.hip) ----
// vblk[2j], vblk[2j+1]: the rows of j's block.  Pattern of D (count with
// Vri null, else fill); LU with partial pivoting of every block of V (at
// most 64 rows), dense column-major at LU + boff[b], row permutation perm;
// *bad += singular blocks (bit 30: an entry of V outside its block); the
// block solve t = V^{-1} x, a no-op once *done.
Err launch_block_vpattern(int n, const int32_t* Acp, const int32_t* Ari, const int32_t* vblk,
                          int32_t* cnt, const int32_t* Vcp, int32_t* Vri, hipStream_t st);
template <class T>
Err launch_block_lu(int nblk, const int32_t* bstart, const int64_t* boff, const int32_t* Vcp,
                    const int32_t* Vri, const T* Vval, T* LU, int32_t* perm, int32_t* bad,
                    hipStream_t st);
template <class T>
Err launch_block_solve(int nblk, const int32_t* bstart, const int64_t* boff, const T* LU,
                       const int32_t* perm, const T* x, T* t, const int32_t* done, hipStream_t st);

// ---- solve (solve.hip) ----

struct TrsvCtl {
    uint32_t ticket;
    uint32_t finished;
    uint32_t epoch;
    uint32_t error;
};

template <class T>
struct BicgState {
    T rho, rho_prev, alpha, omega, beta, ts;
    double bnorm, tol, res, tt;
    int32_t it, maxit, done, flag, half, omega_bad;
    uint32_t red_ticket;
    int32_t pad;
};

template <class T>
Err launch_spmv_csr(int n, int64_t nnz, const int32_t* rp, const int32_t* ci, const T* val,
                    const T* x, T* y, const int32_t* done, hipStream_t st);
// Launch shape of the sync-free triangular solve: waves per workgroup (1, 2,
// 4, 8 or 16; the workgroup owns 64 x waves consecutive rows, one per lane;
// up to 8 waves the LDS has room for twice as many entries per row) and
// whether a wave that found nothing ready sleeps briefly before polling
// again.
struct TrsvTune {
    int backoff = 1;
    int waves = 8;
};
// prefilled: x already holds the not-ready sentinel in every entry (else the
// launch fills it first).
template <class T>
Err launch_trsv(int n, const int32_t* rp, const int32_t* ci, const T* val, int upper, const T* b,
                T* x, TrsvCtl* ctl, const int32_t* done, TrsvTune tune, hipStream_t st,
                bool prefilled = false);
// x = the triangular solve's not-ready sentinel in every entry.
template <class T>
Err launch_fill_sentinel(int n, T* x, hipStream_t st);
template <class T>
Err launch_diag_solve(int n, const int32_t* rp, const int32_t* ci, const T* val, const T* b, T* x,
                      const int32_t* done, hipStream_t st);
// Depth of the triangular dependency DAG (levels) computed on the device.
Err launch_trsv_levels(int n, const int32_t* rp, const int32_t* ci, int upper, int32_t* level,
                       TrsvCtl* ctl, int32_t* maxlevel_dev, hipStream_t st);

// BiCGSTAB stage kernels; every one is a no-op once st->done is set.
template <class T>
struct BicgVecs {
    int n;
    const T* b;
    T *x, *r, *rh, *p, *v, *ph, *s, *sh, *t;
    // when set, bicg_alpha and bicg_xr fill these with the triangular
    // solve's not-ready sentinel: the outputs of the iteration's first and
    // second solve, dead by then, so the solves need no fill launch
    T* clr_a = nullptr;
    T* clr_x = nullptr;
    double* partial;  // reduction scratch (>= 3 * nblocks doubles)
    BicgState<T>* st;
};
template <class T> Err bicg_init(const BicgVecs<T>& V, double tol, int maxit, hipStream_t st);
template <class T> Err bicg_update_p(const BicgVecs<T>& V, hipStream_t st);
template <class T> Err bicg_alpha(const BicgVecs<T>& V, hipStream_t st);
template <class T> Err bicg_s(const BicgVecs<T>& V, hipStream_t st);
template <class T> Err bicg_omega(const BicgVecs<T>& V, hipStream_t st);
template <class T> Err bicg_xr(const BicgVecs<T>& V, hipStream_t st);
template <class T> Err bicg_true_residual(const BicgVecs<T>& V, hipStream_t st);
template <class T> Err bicg_half_fix(const BicgVecs<T>& V, hipStream_t st);

// ---- learned proposer (learned.hip) ----
template <class T>
Err launch_features(int n, const int32_t* Acp, const int32_t* Ari, const T* Aval,
                    const int32_t* Ccp, const int32_t* Cri, float* feat, hipStream_t st);
template <class T>
Err launch_labels(int n, const int32_t* Acp, const int32_t* Ari, const T* Aval, const int32_t* Jcp,
                  const int32_t* Jri, const T* Wval, double tau, float* labels, hipStream_t st);
Err launch_mlp_forward(const float* params, const float* feat, int64_t npairs, float* scores,
                       hipStream_t st);
Err launch_mlp_loss_grad(const float* params, const float* feat, const float* labels,
                         int64_t npairs, float* grad, double* loss_dev, float* scratch,
                         hipStream_t st);
size_t mlp_scratch_floats();
Err launch_adam(float* params, const float* grad, float* m, float* v, int step, float lr,
                hipStream_t st);
// J_j = {j} U {i in C_j : score >= 0} (sigmoid >= 0.5); count / fill.
Err launch_pattern_from_scores(int n, const int32_t* Ccp, const int32_t* Cri,
                               const float* scores, int32_t* cnt, const int32_t* Jcp,
                               int32_t* Jri, hipStream_t st);

// Residual-gated fallback (learned.hip).
Err launch_fallback_count(int n, const int32_t* Jcp, const int32_t* Ccp, const uint8_t* fb,
                          int32_t* cnt, hipStream_t st);
template <class T>
Err launch_fallback_fill(int n, const int32_t* Jcp, const int32_t* Jri, const T* Wval,
                         const int32_t* Ccp, const int32_t* Cri, const uint8_t* fb,
                         const int32_t* Jcp2, int32_t* Jri2, T* Wval2, uint32_t* flags,
                         hipStream_t st);

}  // namespace diaf
