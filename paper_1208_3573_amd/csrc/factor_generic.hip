// Generic column-factoring kernel: one 256-thread workgroup per column,
// any |J_j| up to 256 and up to 8192 gathered entries.
//
// Per column j (paper Sections 2.1, 2.2, 3.1):
//   gather A(:, J_j) from CSC, sort the entries by (row, column) (pairwise
//   merges of the gathered columns, each already sorted by row) to get the
//   shadow R_j and row-ordered access, form the Gram matrix
//   G = B^* B of B = A(R_j, J_j) by sparse merges, then
//   - unit-norm v (first basic algorithm): Cholesky G = L L^*, the seed
//     w0 = G^{-1} b_j^* (V_0 = diagonals), the V pattern, M = L^{-1} B_L^*
//     (the paper's M_j), its top right singular vector v by one-sided
//     Jacobi, and w = L^{-*} M v (the least-squares solution, eq. 2.4);
//   - unit-norm w (second basic algorithm): the seed is the bottom
//     eigenvector of G - b_j^* b_j, and w the bottom eigenvector of
//     G - B_L^* B_L = (B without rows L)^* (B without rows L), both by
//     two-sided cyclic Jacobi; v = (B w) on L;
//   then the phase of (w, v) (diagonal of V real positive), the residual
//   ||B w - v|| in FP64, and the outputs.
// The k x k work matrices live in LDS for small columns and in a per-block
// global slot otherwise.
#include "dcommon.h"
#include "factor_kernels.h"

namespace diaf {

static constexpr int GNT = 512;  // largest workgroup (small size classes use one wave)
static constexpr int kGenMaxK = 256;  // largest |J_j| and l_j of a launch

struct GenLayout {
    size_t oJ, oOff, oKey, oVal, oLrow, oCol, oPos, oRowptr, oR, oRank, oY, oW, oX, oVM, oSig,
        oV, oL, oSel, oRed, oMisc, oMats, total;
    size_t total_lds;  // split layout: bytes of the arrays placed in LDS
    uint32_t in_lds;   // split layout: bit b set = array b (GenArr) lies in LDS
};

// Arrays of a column's working storage.
enum GenArr { GA_J, GA_OFF, GA_KEY, GA_VAL, GA_LROW, GA_COL, GA_POS, GA_ROWPTR, GA_R, GA_RANK,
              GA_Y, GA_W, GA_X, GA_VM, GA_SIG, GA_V, GA_L, GA_SEL, GA_RED, GA_MISC };

__host__ __device__ inline size_t align16(size_t x) { return (x + 15) & ~size_t(15); }

// Working storage of one column.  The key array (sort keys) is dead after
// the shadow is built and is reused for the selection scores.  with_mats =
// number of k x k matrices kept here (1: G, unit-norm v; 3: G, E, Z,
// unit-norm w; 0: in a separate global slot).  lds_budget > 0 splits the
// storage: the small and index arrays read on every step (reduction and
// flag slots, column offsets, the small vectors, the local row of each
// entry, the right-hand sides of the triangular solves, the column and
// position cross references) go, in that order of priority, to LDS while
// they fit in lds_budget bytes, and everything else stays in the global
// slot.
__host__ __device__ inline GenLayout gen_layout(int kcap, int tcap, int tcap2, int lcap, size_t st,
                                                int with_mats, size_t lds_budget = 0)
{
    GenLayout L{};
    size_t o = 0, oi = 0;
    auto take = [&](size_t bytes) { size_t r = o; o = align16(o + bytes); return r; };
    auto takep = [&](int id, size_t bytes) {
        if (lds_budget > 0 && align16(oi + bytes) <= lds_budget) {
            L.in_lds |= 1u << id;
            size_t r = oi;
            oi = align16(oi + bytes);
            return r;
        }
        return take(bytes);
    };
    L.oMisc = takep(GA_MISC, sizeof(double) * 32);
    L.oRed = takep(GA_RED, sizeof(double) * GNT);
    L.oOff = takep(GA_OFF, sizeof(int32_t) * (kcap + 1));
    L.oJ = takep(GA_J, sizeof(int32_t) * kcap);
    L.oL = takep(GA_L, sizeof(int32_t) * lcap);
    L.oSel = takep(GA_SEL, sizeof(int32_t) * lcap);
    L.oW = takep(GA_W, st * kcap);
    L.oVM = takep(GA_VM, st * lcap * lcap);
    L.oSig = takep(GA_SIG, sizeof(double) * lcap);
    L.oV = takep(GA_V, st * lcap);
    L.oLrow = takep(GA_LROW, sizeof(uint16_t) * tcap);
    L.oX = takep(GA_X, st * kcap * (lcap + 1));
    L.oCol = takep(GA_COL, sizeof(uint16_t) * tcap);
    L.oPos = takep(GA_POS, sizeof(uint16_t) * tcap);
    L.oRowptr = takep(GA_ROWPTR, sizeof(uint16_t) * (tcap + 1));
    L.oKey = take(sizeof(uint64_t) * tcap2);
    L.oVal = take(st * tcap);
    L.oR = take(sizeof(int32_t) * tcap);
    L.oRank = take(sizeof(int32_t) * tcap);
    L.oY = take(st * tcap);
    L.oMats = o;
    if (with_mats) take(st * (size_t)with_mats * kcap * kcap);
    L.total = o;
    L.total_lds = oi;
    return L;
}

// misc slots (int view / double view)
enum { MI_T = 0, MI_M, MI_DJ, MI_FLAGS, MI_L, MI_NC, MI_ROT, MI_BEST, MI_Q, MI_EDGE, MI_NIN,
       MI_STAB, MI_DPOS, MI_NULL, MI_RDIG, MI_RREM };
enum { MD_SSTAR = 16, MD_MAXD = 18, MD_GAP, MD_BN2, MD_ERE, MD_EIM, MD_FRO2 };

template <class T>
struct GenCtx {
    int tid, nt;
    int32_t* sJ; int32_t* sOff; uint64_t* sKey; T* sVal; uint16_t* sLrow; uint16_t* sCol;
    uint16_t* sPos; uint16_t* sRowptr; int32_t* sR; int32_t* sRank; T* sY; T* sW; T* sX; T* sVM;
    double* sSig; T* sV; int32_t* sL; int32_t* sSel; double* sScore; double* sRed;
    int* mi; double* md;
    T* G; T* E; T* Z;
    int xld;  // leading dimension of X (= lcap + 1)
};

template <class T>
__device__ inline double block_sum(GenCtx<T>& c, double x)
{
    c.sRed[c.tid] = x;
    __syncthreads();
    for (int s = c.nt / 2; s > 0; s >>= 1) {
        if (c.tid < s) c.sRed[c.tid] += c.sRed[c.tid + s];
        __syncthreads();
    }
    double r = c.sRed[0];
    __syncthreads();
    return r;
}

// Sum of x over the first wave (the other threads pass 0), by a butterfly
// in a fixed order: callers accumulate per lane with stride 64, so the
// result does not depend on the workgroup size.
template <class T>
__device__ inline double wave0_sum(GenCtx<T>& c, double x)
{
    if (c.tid < 64) {
        for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
        if (c.tid == 0) c.sRed[0] = x;
    }
    __syncthreads();
    const double r = c.sRed[0];
    __syncthreads();
    return r;
}

// Inclusive scan of flags[0..cnt) (0/1) into out (ranks; out may be flags),
// returns the total.  Each thread owns a contiguous chunk; the chunk sums are
// scanned within each wave by shuffles and across the (at most 8) waves
// through sRed.
template <class T>
__device__ inline int block_scan_flags(GenCtx<T>& c, const int32_t* flags, int32_t* out, int cnt)
{
    const int chunk = (cnt + c.nt - 1) / c.nt;
    const int b = c.tid * chunk, e = min(cnt, b + chunk);
    int s = 0;
    for (int i = b; i < e; ++i) s += flags[i];
    const int lane = c.tid & 63, wv = c.tid >> 6;
    int x = s;
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    int* wtot = (int*)c.sRed;
    if (lane == 63) wtot[wv] = x;
    __syncthreads();
    int before = 0, tot = 0;
    for (int w = 0; w < (c.nt >> 6); ++w) {
        const int t = wtot[w];
        before += w < wv ? t : 0;
        tot += t;
    }
    int run = before + x - s;
    for (int i = b; i < e; ++i) { run += flags[i]; out[i] = run; }
    __syncthreads();
    return tot;
}

// y = B w over the m local rows (CSR order, deterministic per row).
template <class T>
__device__ inline void bmul(GenCtx<T>& c, int m, const T* w, T* y)
{
    for (int i = c.tid; i < m; i += c.nt) {
        T acc = num<T>::zero();
        for (int p = c.sRowptr[i]; p < c.sRowptr[i + 1]; ++p) {
            int t = c.sPos[p];
            acc += c.sVal[t] * w[c.sCol[t]];
        }
        y[i] = acc;
    }
    __syncthreads();
}

// Entry B(i, a) from the CSR row i (zero if absent).
template <class T>
__device__ inline T bget(const GenCtx<T>& c, int i, int a)
{
    for (int p = c.sRowptr[i]; p < c.sRowptr[i + 1]; ++p) {
        int t = c.sPos[p];
        if (c.sCol[t] == a) return c.sVal[t];
    }
    return num<T>::zero();
}

// In-place lower Cholesky of G (k x k, row-major ld k); zero pivots give a
// zero column.  Sets the rank flag when a pivot^2 (= |R_aa|^2 of B = QR) is
// at most 1e-14 times the largest diagonal entry (squared column norm).
template <class T>
__device__ inline void cholesky(GenCtx<T>& c, T* G, int k)
{
    // column p of the factor is staged in the reduction array (unused here;
    // its GNT doubles hold the k <= 256 entries, complex ones too).  For
    // real values its second half hands the next column (rows >= p + 1, the
    // pivot first) from each step's update to the next step, so the pivot
    // and the column come from LDS, not back from the global slot.
    constexpr bool kHand = !num<T>::is_complex;
    T* lp = (T*)c.sRed;
    double* nx = c.sRed + kGenMaxK;
    if constexpr (kHand)
        for (int i = c.tid; i < k; i += c.nt) nx[i] = num<T>::re(G[i * k]);
    if (c.tid == 0) {
        double mx = 0;
        for (int p = 0; p < k; ++p) mx = fmax(mx, num<T>::re(G[p * k + p]));
        c.md[MD_MAXD] = mx;
    }
    __syncthreads();
    const double maxd = c.md[MD_MAXD];
    const int lane = c.tid & 63, wv = c.tid >> 6, nw = c.nt >> 6;
    for (int p = 0; p < k; ++p) {
        // every thread forms the pivot from the updated diagonal; thread 0
        // stores it after the barrier, once all have read the diagonal
        double d;
        if constexpr (kHand) d = nx[p];
        else d = num<T>::re(G[p * k + p]);
        double piv = 0.0;
        if (d > 1e-30 * maxd && isfinite(d)) piv = sqrt(d);
        for (int i = p + 1 + c.tid; i < k; i += c.nt) {
            T gi;
            if constexpr (kHand) gi = nx[i];
            else gi = G[i * k + p];
            const T v = piv > 0.0 ? num<T>::div(gi, piv) : num<T>::zero();
            G[i * k + p] = v;
            lp[i] = v;
        }
        __syncthreads();
        if (c.tid == 0) {
            if (!(d > 1e-14 * maxd)) c.mi[MI_FLAGS] |= DIAF_FLAG_RANK_DEFICIENT;
            G[p * k + p] = num<T>::mk(piv);
        }
        // trailing update of the lower triangle: each wave takes four rows
        // at a time and lanes sweep the columns q <= i, 64 per pass, with the
        // four rows' loads of a pass issued before their stores (a load
        // issued after a store waits for it too)
        for (int i0 = p + 1 + 4 * wv; i0 < k; i0 += 4 * nw) {
            const int imax = min(i0 + 3, k - 1);
            for (int q = p + 1 + lane; q - lane <= imax; q += 64) {
                T g[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int i = i0 + r;
                    g[r] = (i < k && q <= i) ? G[i * k + q] : num<T>::zero();
                }
                const T lq = q <= imax ? num<T>::conj(lp[q]) : num<T>::zero();
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int i = i0 + r;
                    if (i < k && q <= i) {
                        const T v = g[r] - lp[i] * lq;
                        G[i * k + q] = v;
                        if constexpr (kHand)
                            if (q == p + 1) nx[i] = v;
                    }
                }
            }
        }
        __syncthreads();
    }
}

// Solve L X = X (forward) for nr right-hand sides stored X[a * xld + t].
// X(p, :) is final once step p starts.  For few right-hand sides every
// thread forms x_p = X(p, :) / L(p, p) itself (the same value each time), so
// a step needs one barrier, and the scaled rows are written back at the end;
// for many, one pass scales row p first (two barriers a step, one division
// per entry).
template <class T>
__device__ inline void lsolve(GenCtx<T>& c, const T* Lf, int k, T* X, int nr)
{
    const bool few = nr <= 8;
    for (int p = 0; p < k; ++p) {
        const double d = num<T>::re(Lf[p * k + p]);
        if (!few) {
            for (int t = c.tid; t < nr; t += c.nt)
                X[p * c.xld + t] = d > 0.0 ? num<T>::div(X[p * c.xld + t], d) : num<T>::zero();
            __syncthreads();
        }
        const int rem = k - p - 1;
        for (int idx = c.tid; idx < rem * nr; idx += c.nt) {
            const int i = p + 1 + idx / nr, t = idx % nr;
            T xp = X[p * c.xld + t];
            if (few) xp = d > 0.0 ? num<T>::div(xp, d) : num<T>::zero();
            X[i * c.xld + t] -= Lf[i * k + p] * xp;
        }
        __syncthreads();
    }
    if (few) {
        for (int idx = c.tid; idx < k * nr; idx += c.nt) {
            const int p = idx / nr, t = idx % nr;
            const double d = num<T>::re(Lf[p * k + p]);
            X[p * c.xld + t] = d > 0.0 ? num<T>::div(X[p * c.xld + t], d) : num<T>::zero();
        }
        __syncthreads();
    }
}

// Solve L^* X = X (backward), in the same way.
template <class T>
__device__ inline void lhsolve(GenCtx<T>& c, const T* Lf, int k, T* X, int nr)
{
    const bool few = nr <= 8;
    for (int p = k - 1; p >= 0; --p) {
        const double d = num<T>::re(Lf[p * k + p]);
        if (!few) {
            for (int t = c.tid; t < nr; t += c.nt)
                X[p * c.xld + t] = d > 0.0 ? num<T>::div(X[p * c.xld + t], d) : num<T>::zero();
            __syncthreads();
        }
        for (int idx = c.tid; idx < p * nr; idx += c.nt) {
            const int i = idx / nr, t = idx % nr;
            T xp = X[p * c.xld + t];
            if (few) xp = d > 0.0 ? num<T>::div(xp, d) : num<T>::zero();
            X[i * c.xld + t] -= num<T>::conj(Lf[p * k + i]) * xp;
        }
        __syncthreads();
    }
    if (few) {
        for (int idx = c.tid; idx < k * nr; idx += c.nt) {
            const int p = idx / nr, t = idx % nr;
            const double d = num<T>::re(Lf[p * k + p]);
            X[p * c.xld + t] = d > 0.0 ? num<T>::div(X[p * c.xld + t], d) : num<T>::zero();
        }
        __syncthreads();
    }
}

// Round-robin pairing of nplayers (even) players in round r, pair i.
__device__ inline void rr_pair(int np, int r, int i, int& a, int& b)
{
    if (i == 0) { a = np - 1; b = r; }
    else { a = (r + i) % (np - 1); b = (r - i + (np - 1)) % (np - 1); }
    if (a > b) { int t = a; a = b; b = t; }
}

// Rotation (c, s, ec) that orthogonalises / diagonalises the pair with
// diagonal entries al, be and off-diagonal g:
//   J = [[c, s], [-s ec, c ec]],  ec = conj(g) / |g|.
template <class T>
__device__ inline void jrot(double al, double be, T g, double& cs, double& sn, T& ec)
{
    double ag = num<T>::abs(g);
    double zeta = (be - al) / (2.0 * ag);
    double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
    cs = 1.0 / sqrt(1.0 + t * t);
    sn = cs * t;
    ec = num<T>::div(num<T>::conj(g), ag);
}

// One-sided Jacobi on the columns of M (k x l, stored X[a * xld + t]);
// VM (l x l, row-major ld l) accumulates the rotations.
template <class T>
__device__ inline void jacobi_onesided(GenCtx<T>& c, T* M, int k, int l, T* VM)
{
    for (int idx = c.tid; idx < l * l; idx += c.nt)
        VM[idx] = (idx / l == idx % l) ? num<T>::one() : num<T>::zero();
    const int np = l + (l & 1);
    __shared__ double s_c[128], s_s[128];
    __shared__ T s_e[128];
    __shared__ int s_p[128], s_q[128];
    for (int sweep = 0; sweep < 40; ++sweep) {
        if (c.tid == 0) c.mi[MI_ROT] = 0;
        __syncthreads();
        for (int r = 0; r < np - 1; ++r) {
            for (int i = c.tid; i < np / 2; i += c.nt) {
                int a, b;
                rr_pair(np, r, i, a, b);
                s_p[i] = a; s_q[i] = b; s_s[i] = 0.0; s_c[i] = 1.0;
                if (b < l) {
                    double al = 0, be = 0;
                    T g = num<T>::zero();
                    for (int e = 0; e < k; ++e) {
                        T xa = M[e * c.xld + a], xb = M[e * c.xld + b];
                        al += num<T>::abs2(xa);
                        be += num<T>::abs2(xb);
                        g += num<T>::cmul(xa, xb);
                    }
                    double ag = num<T>::abs(g);
                    if (al > 0.0 && be > 0.0 && ag > 1e-15 * sqrt(al) * sqrt(be)) {
                        double cs, sn; T ec;
                        jrot<T>(al, be, g, cs, sn, ec);
                        s_c[i] = cs; s_s[i] = sn; s_e[i] = ec;
                        c.mi[MI_ROT] = 1;
                    }
                }
            }
            __syncthreads();
            const int npair = np / 2;
            for (int idx = c.tid; idx < npair * (k + l); idx += c.nt) {
                int i = idx % npair, e = idx / npair;
                if (s_s[i] == 0.0) continue;
                int a = s_p[i], b = s_q[i];
                double cs = s_c[i], sn = s_s[i];
                T ec = s_e[i];
                T* pa; T* pb;
                if (e < k) { pa = &M[e * c.xld + a]; pb = &M[e * c.xld + b]; }
                else { int f = e - k; pa = &VM[f * l + a]; pb = &VM[f * l + b]; }
                T u = *pa, w = *pb;
                *pa = cs * u - sn * (ec * w);
                *pb = sn * u + cs * (ec * w);
            }
            __syncthreads();
        }
        if (c.mi[MI_ROT] == 0) break;
        __syncthreads();
    }
    __syncthreads();
}

// Two-sided cyclic Jacobi on the Hermitian E (k x k, row-major ld k);
// Z accumulates the eigenvectors (columns).
template <class T>
__device__ inline void jacobi_eig(GenCtx<T>& c, T* E, T* Z, int k)
{
    for (int idx = c.tid; idx < k * k; idx += c.nt)
        Z[idx] = (idx / k == idx % k) ? num<T>::one() : num<T>::zero();
    if (c.tid == 0) {
        double mx = 0;
        for (int p = 0; p < k; ++p) mx = fmax(mx, fabs(num<T>::re(E[p * k + p])));
        c.md[MD_MAXD] = mx;
    }
    __syncthreads();
    const double scale = c.md[MD_MAXD];
    const int np = k + (k & 1);
    const int npair = np / 2;
    __shared__ double s_c[128], s_s[128];
    __shared__ T s_e[128];
    __shared__ int s_p[128], s_q[128];
    for (int sweep = 0; sweep < 40; ++sweep) {
        if (c.tid == 0) c.mi[MI_ROT] = 0;
        __syncthreads();
        for (int r = 0; r < np - 1; ++r) {
            for (int i = c.tid; i < npair; i += c.nt) {
                int a, b;
                rr_pair(np, r, i, a, b);
                s_p[i] = a; s_q[i] = b; s_s[i] = 0.0; s_c[i] = 1.0;
                if (b < k) {
                    double al = num<T>::re(E[a * k + a]), be = num<T>::re(E[b * k + b]);
                    T g = E[a * k + b];
                    double ag = num<T>::abs(g);
                    if (ag > 1e-15 * sqrt(fabs(al)) * sqrt(fabs(be)) && ag > 1e-300 + 1e-30 * scale) {
                        double cs, sn; T ec;
                        jrot<T>(al, be, g, cs, sn, ec);
                        s_c[i] = cs; s_s[i] = sn; s_e[i] = ec;
                        c.mi[MI_ROT] = 1;
                    }
                }
            }
            __syncthreads();
            // rows: E[[a,b], :] <- J^* E[[a,b], :]
            for (int idx = c.tid; idx < npair * k; idx += c.nt) {
                int i = idx % npair, e = idx / npair;
                if (s_s[i] == 0.0) continue;
                int a = s_p[i], b = s_q[i];
                double cs = s_c[i], sn = s_s[i];
                T ecc = num<T>::conj(s_e[i]);
                T u = E[a * k + e], w = E[b * k + e];
                E[a * k + e] = cs * u - sn * (ecc * w);
                E[b * k + e] = sn * u + cs * (ecc * w);
            }
            __syncthreads();
            // columns: E[:, [a,b]] <- E[:, [a,b]] J, Z likewise
            for (int idx = c.tid; idx < npair * 2 * k; idx += c.nt) {
                int i = idx % npair, e = idx / npair;
                if (s_s[i] == 0.0) continue;
                int a = s_p[i], b = s_q[i];
                double cs = s_c[i], sn = s_s[i];
                T ec = s_e[i];
                T* M = e < k ? E : Z;
                int row = e < k ? e : e - k;
                T u = M[row * k + a], w = M[row * k + b];
                M[row * k + a] = cs * u - sn * (ec * w);
                M[row * k + b] = sn * u + cs * (ec * w);
            }
            __syncthreads();
        }
        if (c.mi[MI_ROT] == 0) break;
        __syncthreads();
    }
    __syncthreads();
}

// The q-th largest (1-based) of the admissible scores sScore[0..m) (those
// not below zero), found by radix selection on their bit patterns, which
// order as the values for non-negative doubles: 8 passes over 8-bit digits
// from the top, each counting the candidates that match the digits fixed so
// far into 256 bins and fixing the digit in which the q-th falls.  The
// caller guarantees more than q candidates.
template <class T>
__device__ inline double kth_largest_score(GenCtx<T>& c, int m, int q)
{
    int* hist = (int*)c.sRed;  // 256 counters (sRed holds GNT doubles)
    uint64_t prefix = 0, mask = 0;
    int rem = q;
    for (int shift = 56; shift >= 0; shift -= 8) {
        for (int b = c.tid; b < 256; b += c.nt) hist[b] = 0;
        __syncthreads();
        for (int t = c.tid; t < m; t += c.nt) {
            const double s = c.sScore[t];
            if (s < 0.0) continue;
            const uint64_t key = (uint64_t)__double_as_longlong(s) & 0x7fffffffffffffffull;
            if ((key & mask) == prefix) atomicAdd(&hist[(key >> shift) & 255], 1);
        }
        __syncthreads();
        if (c.tid < 64) {
            // lane l holds bins 255 - 4l down to 252 - 4l; counts accumulate
            // from the top bin down
            const int lane = c.tid;
            int h[4], loc = 0;
            for (int r = 0; r < 4; ++r) { h[r] = hist[255 - 4 * lane - r]; loc += h[r]; }
            int x = loc;
            for (int o = 1; o < 64; o <<= 1) {
                const int y = __shfl_up(x, o);
                if (lane >= o) x += y;
            }
            const int excl = x - loc;
            if (excl < rem && rem <= x) {
                int run = excl, r = 0;
                while (r < 3 && run + h[r] < rem) { run += h[r]; ++r; }
                c.mi[MI_RDIG] = 255 - 4 * lane - r;
                c.mi[MI_RREM] = rem - run;
            }
        }
        __syncthreads();
        prefix |= (uint64_t)(uint32_t)c.mi[MI_RDIG] << shift;
        mask |= 255ull << shift;
        rem = c.mi[MI_RREM];
    }
    return __longlong_as_double((long long)prefix);
}

// Top-q selection with the 1e-10 tie band over the m local rows;
// sScore[i] = |(B w0)_i| for admissible rows and -1 otherwise (rows are in
// ascending order).  With s* the q-th largest score, every row above
// s*(1 + 1e-10) is taken and the rest of the q come from the band
// [s*(1 - 1e-10), s*(1 + 1e-10)] in ascending row order.  Writes the chosen
// local rows, ascending, to sL from index 1 (index 0 holds the diagonal) and
// returns the count.  sRank is free here and holds the flags and ranks.
template <class T>
__device__ inline int select_topk(GenCtx<T>& c, int m, int nc, int q)
{
    if (q <= 0) return 0;
    int32_t* fl = c.sRank;
    if (c.tid == 0) { c.mi[MI_EDGE] = 0; c.mi[MI_RDIG] = 0; c.mi[MI_RREM] = 1; }
    __syncthreads();
    if (nc <= q) {
        for (int t = c.tid; t < m; t += c.nt) fl[t] = c.sScore[t] >= 0.0;
        __syncthreads();
    } else {
        const double ss = kth_largest_score(c, m, q);
        const double hi = ss * (1.0 + 1e-10), lo = ss * (1.0 - 1e-10);
        int above = 0;
        for (int t = c.tid; t < m; t += c.nt) {
            const double s = c.sScore[t];
            const bool adm = s >= 0.0;
            above += adm && s > hi;
            fl[t] = adm && s >= lo && s <= hi;
            if (adm && ss > 0.0 && (fabs(s - hi) <= 1e-12 * ss || fabs(s - lo) <= 1e-12 * ss))
                c.mi[MI_EDGE] = 1;
        }
        const int need = q - (int)block_sum(c, (double)above);
        block_scan_flags(c, fl, fl, m);  // band rank of each row
        for (int t = c.tid; t < m; t += c.nt) {
            const double s = c.sScore[t];
            const bool adm = s >= 0.0;
            const bool band = adm && s >= lo && s <= hi;
            fl[t] = (adm && s > hi) || (band && fl[t] <= need);
        }
        __syncthreads();
        if (c.tid == 0 && c.mi[MI_EDGE]) c.mi[MI_FLAGS] |= DIAF_FLAG_TIE_EDGE;
    }
    const int cnt = block_scan_flags(c, fl, fl, m);
    for (int t = c.tid; t < m; t += c.nt) {
        const int r = fl[t], p = t ? fl[t - 1] : 0;
        if (r != p && r <= q) c.sL[r] = t;
    }
    __syncthreads();
    return cnt < q ? cnt : q;
}

template <class T>
__device__ int find_local_row(const GenCtx<T>& c, int m, int row)
{
    int lo = 0, hi = m - 1;
    while (lo <= hi) {
        int mid = (lo + hi) >> 1;
        int v = c.sR[mid];
        if (v == row) return mid;
        if (v < row) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

template <class T>
__device__ void factor_one_column(const FactorArgs<T>& A, int j, GenCtx<T>& c)
{
    const int tid = c.tid;
    const int jb = A.Jcp[j];
    const int k = A.Jcp[j + 1] - jb;
    // ---- 1. J_j and per-column offsets ----
    if (tid == 0) { c.mi[MI_FLAGS] = 0; c.sOff[0] = 0; }
    for (int a = tid; a < k; a += c.nt) {
        int col = A.Jri[jb + a];
        c.sJ[a] = col;
        c.sOff[a + 1] = A.Acp[col + 1] - A.Acp[col];
    }
    __syncthreads();
    const int Tn = block_scan_flags(c, c.sOff + 1, c.sOff + 1, k);
    // ---- 2. gather ----
    // Keys (row << 32) | (a << 16) | t for the entry at gather position t,
    // which comes from A(:, J_j(a)) (t and a < 65536, the u16 cross
    // references); gather positions follow ascending a, so this orders by
    // (row, t), and every key is unique.  The gather is k runs sorted by row
    // (one per column of A), merged pairwise in ceil(log2 k) rounds; the
    // right-hand-side array, unused until the V pattern, is the second
    // buffer, and the gather writes into the one the last round leaves in
    // sKey.
    int rounds = 0;
    while ((1 << rounds) < k) ++rounds;
    uint64_t* ybuf = (uint64_t*)c.sY;
    uint64_t* gbuf = (rounds & 1) ? ybuf : c.sKey;
    for (int t = tid; t < Tn; t += c.nt) {
        int lo = 0, hi = k - 1;  // largest a with sOff[a] <= t
        while (lo < hi) {
            int mid = (lo + hi + 1) >> 1;
            if (c.sOff[mid] <= t) lo = mid; else hi = mid - 1;
        }
        int a = lo;
        int p = A.Acp[c.sJ[a]] + (t - c.sOff[a]);
        gbuf[t] = ((uint64_t)(uint32_t)A.Ari[p] << 32) | ((uint32_t)a << 16) | (uint32_t)t;
        c.sVal[t] = A.Aval[p];
        c.sCol[t] = a;
    }
    __syncthreads();
    // ---- 3. merge rounds: sort by (row, t) ----
    for (int r = 0; r < rounds; ++r) {
        const uint64_t* src = ((rounds - r) & 1) ? ybuf : c.sKey;
        uint64_t* dst = ((rounds - r) & 1) ? c.sKey : ybuf;
        for (int t = tid; t < Tn; t += c.nt) {
            const uint64_t key = src[t];
            // merged groups of 2^r runs; this entry's is (its run) >> r
            const int g = (int)((key >> 16) & 0xffff) >> r, h = g ^ 1;
            const int gs = c.sOff[g << r];
            if ((h << r) >= k) {
                dst[t] = key;  // no partner group this round
                continue;
            }
            const int hs = c.sOff[h << r], he = c.sOff[min((h + 1) << r, k)];
            int lo = hs, hi = he;  // first partner key above this one
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (src[mid] < key) lo = mid + 1; else hi = mid;
            }
            dst[min(gs, hs) + (t - gs) + (lo - hs)] = key;
        }
        __syncthreads();
    }
    // ---- 4. shadow rows and CSR/CSC cross references ----
    for (int i = tid; i < Tn; i += c.nt)
        c.sRank[i] = (i == 0 || (c.sKey[i] >> 32) != (c.sKey[i - 1] >> 32)) ? 1 : 0;
    __syncthreads();
    int m = block_scan_flags(c, c.sRank, c.sRank, Tn);
    for (int i = tid; i < Tn; i += c.nt) {
        int lr = c.sRank[i] - 1;
        int t = (int)(c.sKey[i] & 0xffff);
        c.sPos[i] = t;
        c.sLrow[t] = lr;
        if (i == 0 || (c.sKey[i] >> 32) != (c.sKey[i - 1] >> 32)) {
            c.sR[lr] = (int)(c.sKey[i] >> 32);
            c.sRowptr[lr] = i;
        }
    }
    if (tid == 0) c.sRowptr[m] = Tn;
    __syncthreads();
    if (tid == 0) c.mi[MI_DJ] = find_local_row(c, m, j);
    __syncthreads();
    const int dj = c.mi[MI_DJ];
    // ||B||_F
    {
        double s = 0;
        if (tid < 64)
            for (int t = tid; t < Tn; t += 64) s += num<T>::abs2(c.sVal[t]);
        double bn2 = wave0_sum(c, s);
        if (tid == 0) c.md[MD_BN2] = bn2;
    }
    const int lmax = A.lmax;
    if (dj < 0) {
        for (int a = tid; a < k; a += c.nt) A.Wval[jb + a] = num<T>::zero();
        for (int t = tid; t < lmax; t += c.nt) {
            A.Vrows[(size_t)j * lmax + t] = -1;
            A.Vvals[(size_t)j * lmax + t] = num<T>::zero();
        }
        if (tid == 0) {
            A.rcol[j] = 0.0;
            A.bnorm[j] = sqrt(c.md[MD_BN2]);
            A.flags[j] = DIAF_FLAG_NO_DIAG_ROW;
            A.lcount[j] = 0;
        }
        __syncthreads();
        return;
    }
    // ---- 5. Gram matrix G = B^* B by sparse merges ----
    T* G = c.G;
    for (int idx = tid; idx < k * k; idx += c.nt) {
        int a = idx / k, b = idx % k;
        if (b < a) continue;
        int pa = c.sOff[a], ea = c.sOff[a + 1], pb = c.sOff[b], eb = c.sOff[b + 1];
        T acc = num<T>::zero();
        if (A.gram_fp32) {
            // variant: products and sums in FP32
            float ax = 0.f, ay = 0.f;
            while (pa < ea && pb < eb) {
                int ra = c.sLrow[pa], rb = c.sLrow[pb];
                if (ra == rb) {
                    T va = c.sVal[pa], vb = c.sVal[pb];
                    T pr = num<T>::cmul(va, vb);
                    ax += (float)num<T>::re(pr);
                    ay += (float)num<T>::im(pr);
                    ++pa; ++pb;
                } else if (ra < rb) ++pa; else ++pb;
            }
            if constexpr (num<T>::is_complex) acc = T{(double)ax, (double)ay};
            else acc = (double)ax;
        } else {
            while (pa < ea && pb < eb) {
                int ra = c.sLrow[pa], rb = c.sLrow[pb];
                if (ra == rb) { acc += num<T>::cmul(c.sVal[pa], c.sVal[pb]); ++pa; ++pb; }
                else if (ra < rb) ++pa;
                else ++pb;
            }
        }
        G[a * k + b] = acc;
        G[b * k + a] = num<T>::conj(acc);
    }
    __syncthreads();

    // ---- 6. V pattern ----
    const bool topk =
        (A.vrule == V_TOPK_LOWER || A.vrule == V_TOPK_UPPER || A.vrule == V_TOPK_BLOCK);
    const bool lev = A.mode == 0 && (A.vrule == V_LEV_LOWER || A.vrule == V_LEV_UPPER);
    const bool lowerrule = A.vrule == V_TOPK_LOWER || A.vrule == V_LEV_LOWER;
    int l = 0;
    if (A.mode == 0) cholesky(c, G, k);
    if (topk || lev) {
        T* E = c.E; T* Z = c.Z;
        if (lev) {
            // Section 3.1's rule: the score of row i is the norm of its column
            // of Q^*, ||L^{-1} b_i^*|| with G = L L^* (rows in batches of
            // xld columns of X; non-admissible rows are scored and dropped)
            const int nbmax = c.xld;
            for (int base = 0; base < m; base += nbmax) {
                const int nb = min(nbmax, m - base);
                for (int idx = tid; idx < k * nb; idx += c.nt) {
                    const int a = idx / nb, t = idx % nb;
                    c.sX[a * c.xld + t] = num<T>::conj(bget(c, base + t, a));
                }
                __syncthreads();
                lsolve(c, G, k, c.sX, nb);
                for (int t = tid; t < nb; t += c.nt) {
                    double h = 0;
                    for (int a = 0; a < k; ++a) h += num<T>::abs2(c.sX[a * c.xld + t]);
                    c.sY[base + t] = num<T>::mk(sqrt(h));
                }
                __syncthreads();
            }
        } else if (A.mode == 0) {
            // seed w0 = G^{-1} b_j^*  (V_0 = diagonals: the SPAI column)
            for (int a = tid; a < k; a += c.nt) c.sX[a * c.xld] = num<T>::zero();
            __syncthreads();
            for (int p = c.sRowptr[dj] + tid; p < c.sRowptr[dj + 1]; p += c.nt) {
                int t = c.sPos[p];
                c.sX[c.sCol[t] * c.xld] = num<T>::conj(c.sVal[t]);
            }
            __syncthreads();
            lsolve(c, G, k, c.sX, 1);
            lhsolve(c, G, k, c.sX, 1);
            for (int a = tid; a < k; a += c.nt) c.sW[a] = c.sX[a * c.xld];
            __syncthreads();
        } else {
            // seed: bottom eigenvector of G - b_j^* b_j
            for (int idx = tid; idx < k * k; idx += c.nt) {
                int a = idx / k, b = idx % k;
                E[idx] = G[idx] - num<T>::cmul(bget(c, dj, a), bget(c, dj, b));
            }
            __syncthreads();
            jacobi_eig(c, E, Z, k);
            if (tid == 0) {
                int lo = 0;
                for (int p = 1; p < k; ++p)
                    if (num<T>::re(E[p * k + p]) < num<T>::re(E[lo * k + lo])) lo = p;
                c.mi[MI_BEST] = lo;
            }
            __syncthreads();
            const int lo = c.mi[MI_BEST];
            for (int a = tid; a < k; a += c.nt) c.sW[a] = Z[a * k + lo];
            __syncthreads();
        }
        if (topk) bmul(c, m, c.sW, c.sY);
        // scores of the admissible rows (ascending row order); -1 elsewhere
        int ncl = 0;
        for (int i = tid; i < m; i += c.nt) {
            int gi = c.sR[i];
            int adm = A.vrule == V_TOPK_BLOCK
                          ? (gi != j && gi >= A.vblk[2 * j] && gi < A.vblk[2 * j + 1])
                          : (lowerrule ? (gi > j) : (gi < j));
            c.sScore[i] = adm ? num<T>::abs(c.sY[i]) : -1.0;
            ncl += adm;
        }
        int nc = (int)block_sum(c, (double)ncl);
        int lj = A.vcount < 1 ? 1 : A.vcount;
        if (lj > 1 + nc) lj = 1 + nc;
        if (A.mode == 1) {
            int cap = m - k > 1 ? m - k : 1;
            if (lj > cap) lj = cap;
        }
        if (lj > lmax) lj = lmax;
        if (tid == 0) c.sL[0] = dj;
        __syncthreads();
        int nsel = select_topk(c, m, nc, lj - 1);
        l = 1 + nsel;
    } else {
        if (tid == 0) {
            int cnt = 0;
            if (A.vrule == V_DIAG) {
                c.sL[cnt++] = dj;
            } else if (A.vrule == V_GS_UPPER || A.vrule == V_GS_LOWER) {
                for (int p = A.Acp[j]; p < A.Acp[j + 1]; ++p) {
                    int gi = A.Ari[p];
                    bool keep = gi == j || (A.vrule == V_GS_UPPER ? gi < j : gi > j);
                    if (!keep) continue;
                    int lr = find_local_row(c, m, gi);
                    if (lr >= 0 && cnt < lmax) c.sL[cnt++] = lr;
                }
            } else {
                for (int p = A.Vcp_in[j]; p < A.Vcp_in[j + 1]; ++p) {
                    int lr = find_local_row(c, m, A.Vri_in[p]);
                    if (lr >= 0 && cnt < lmax) c.sL[cnt++] = lr;
                }
            }
            c.mi[MI_L] = cnt;
        }
        __syncthreads();
        l = c.mi[MI_L];
        __syncthreads();
    }

    // ---- 7. final solve on (J_j, L_j) ----
    if (A.mode == 0) {
        // M = L^{-1} B_L^*  (k x l)
        for (int idx = tid; idx < k * l; idx += c.nt) {
            int a = idx / l, t = idx % l;
            c.sX[a * c.xld + t] = num<T>::conj(bget(c, c.sL[t], a));
        }
        __syncthreads();
        lsolve(c, G, k, c.sX, l);
        jacobi_onesided(c, c.sX, k, l, c.sVM);
        for (int t = tid; t < l; t += c.nt) {
            double s = 0;
            for (int a = 0; a < k; ++a) s += num<T>::abs2(c.sX[a * c.xld + t]);
            c.sSig[t] = sqrt(s);
        }
        __syncthreads();
        if (tid == 0) {
            int best = 0;
            for (int t = 1; t < l; ++t) if (c.sSig[t] > c.sSig[best]) best = t;
            double s1 = c.sSig[best], s2 = 0;
            for (int t = 0; t < l; ++t) if (t != best && c.sSig[t] > s2) s2 = c.sSig[t];
            double gap = (l >= 2 && s1 > 0) ? (s1 * s1 - s2 * s2) / (s1 * s1) : 1.0;
            if (gap < 1e-6) c.mi[MI_FLAGS] |= DIAF_FLAG_GAP_DEGENERATE;
            c.mi[MI_BEST] = best;
        }
        __syncthreads();
        const int best = c.mi[MI_BEST];
        for (int t = tid; t < l; t += c.nt) c.sV[t] = c.sVM[t * l + best];
        // u = M v = (rotated M)(:, best); w = L^{-*} u
        for (int a = tid; a < k; a += c.nt) c.sX[a * c.xld + l] = c.sX[a * c.xld + best];
        __syncthreads();
        for (int a = tid; a < k; a += c.nt) c.sX[a * c.xld] = c.sX[a * c.xld + l];
        __syncthreads();
        lhsolve(c, G, k, c.sX, 1);
        for (int a = tid; a < k; a += c.nt) c.sW[a] = c.sX[a * c.xld];
        __syncthreads();
    } else {
        T* E = c.E; T* Z = c.Z;
        for (int idx = tid; idx < k * k; idx += c.nt) {
            int a = idx / k, b = idx % k;
            T acc = G[idx];
            for (int t = 0; t < l; ++t) acc -= num<T>::cmul(bget(c, c.sL[t], a), bget(c, c.sL[t], b));
            E[idx] = acc;
        }
        __syncthreads();
        jacobi_eig(c, E, Z, k);
        // ||Bh||_F^2 over the entries of B outside the rows of L (Bh = B
        // without those rows; its Gram matrix is E)
        {
            double s2 = 0.0;
            if (tid < 64)
                for (int t = tid; t < Tn; t += 64) {
                    const int lr = c.sLrow[t];
                    bool inL = false;
                    for (int q = 0; q < l; ++q) inL |= c.sL[q] == lr;
                    if (!inL) s2 += num<T>::abs2(c.sVal[t]);
                }
            const double fro2 = wave0_sum(c, s2);
            if (tid == 0) c.md[MD_FRO2] = fro2;
        }
        if (tid == 0) {
            int lo = 0, hi = 0;
            for (int p = 1; p < k; ++p) {
                double d = num<T>::re(E[p * k + p]);
                if (d < num<T>::re(E[lo * k + lo])) lo = p;
                if (d > num<T>::re(E[hi * k + hi])) hi = p;
            }
            double l1 = num<T>::re(E[lo * k + lo]), lmx = num<T>::re(E[hi * k + hi]);
            double l2 = INFINITY;
            for (int p = 0; p < k; ++p)
                if (p != lo) l2 = fmin(l2, num<T>::re(E[p * k + p]));
            double gap = (k >= 2 && lmx > 0) ? (l2 - l1) / lmx : 1.0;
            c.mi[MI_BEST] = lo;
            c.mi[MI_NULL] = 0;
            // A null space N of Bh of dimension >= 2 (eigenvalues of E at
            // most 1e-14 ||Bh||_F^2): take the unit w in N that maximises
            // |(B w)_j|, i.e. P_N b^* normalised with b = row j of B, unless
            // P_N b^* is negligible (then every w in N gives v_jj ~ 0).
            const double thr = 1e-14 * c.md[MD_FRO2];
            int nnull = 0;
            double lin = 0.0, lout = INFINITY;
            for (int p = 0; p < k; ++p) {
                const double d = num<T>::re(E[p * k + p]);
                if (d <= thr) { ++nnull; lin = fmax(lin, d); }
                else lout = fmin(lout, d);
            }
            if (nnull >= 2) {
                T* bj = c.sX;  // conj(B(j, :)) in column 0 of X
                double bn2 = 0.0;
                for (int a = 0; a < k; ++a) bj[a * c.xld] = num<T>::zero();
                for (int pp = c.sRowptr[dj]; pp < c.sRowptr[dj + 1]; ++pp) {
                    const int t = c.sPos[pp];
                    bj[c.sCol[t] * c.xld] = num<T>::conj(c.sVal[t]);
                    bn2 += num<T>::abs2(c.sVal[t]);
                }
                for (int a = 0; a < k; ++a) c.sW[a] = num<T>::zero();
                for (int p = 0; p < k; ++p) {
                    if (!(num<T>::re(E[p * k + p]) <= thr)) continue;
                    T coef = num<T>::zero();  // z_p^* b^*
                    for (int a = 0; a < k; ++a) coef += num<T>::cmul(Z[a * k + p], bj[a * c.xld]);
                    for (int a = 0; a < k; ++a) c.sW[a] += Z[a * k + p] * coef;
                }
                double un2 = 0.0;
                for (int a = 0; a < k; ++a) un2 += num<T>::abs2(c.sW[a]);
                if (un2 > 1e-16 * bn2 && un2 > 0.0) {
                    const double inv = 1.0 / sqrt(un2);
                    for (int a = 0; a < k; ++a) c.sW[a] = c.sW[a] * inv;
                    c.mi[MI_NULL] = 1;
                    c.mi[MI_FLAGS] |= DIAF_FLAG_NULL_CHOICE;
                    gap = (lout < INFINITY && lmx > 0) ? (lout - lin) / lmx : 1.0;
                }
            }
            if (gap < 1e-6) c.mi[MI_FLAGS] |= DIAF_FLAG_GAP_DEGENERATE;
        }
        __syncthreads();
        const int lo = c.mi[MI_BEST];
        if (!c.mi[MI_NULL])
            for (int a = tid; a < k; a += c.nt) c.sW[a] = Z[a * k + lo];
        __syncthreads();
        bmul(c, m, c.sW, c.sY);
        for (int t = tid; t < l; t += c.nt) c.sV[t] = c.sY[c.sL[t]];
        __syncthreads();
    }

    // ---- 8. phase, residual, outputs ----
    if (tid == 0) {
        double vn2 = 0;
        for (int t = 0; t < l; ++t) vn2 += num<T>::abs2(c.sV[t]);
        double vn = sqrt(vn2);
        int dpos = -1;
        for (int t = 0; t < l; ++t) if (c.sL[t] == dj) dpos = t;
        int piv = 0;
        if (dpos >= 0 && num<T>::abs(c.sV[dpos]) >= 1e-8 * vn) {
            piv = dpos;
        } else {
            double bestv = -1.0;
            int bestrow = 0;
            for (int t = 0; t < l; ++t) {
                double a = num<T>::abs(c.sV[t]);
                int gr = c.sR[c.sL[t]];
                if (a > bestv || (a == bestv && gr < bestrow)) { bestv = a; bestrow = gr; piv = t; }
            }
        }
        T ph = num<T>::one();
        if (!num<T>::iszero(c.sV[piv])) ph = unit_conj_phase(c.sV[piv]);
        for (int t = 0; t < l; ++t) c.sV[t] = ph * c.sV[t];
        for (int a = 0; a < k; ++a) c.sW[a] = ph * c.sW[a];
        // Section 3.2 applies to unit-norm v with a triangular V
        const bool vtri = A.vrule == V_DIAG || A.vrule == V_GS_UPPER || A.vrule == V_GS_LOWER ||
                          A.vrule == V_TOPK_UPPER || A.vrule == V_TOPK_LOWER ||
                          A.vrule == V_LEV_UPPER || A.vrule == V_LEV_LOWER;
        const bool stab = A.mode == 0 && A.stab_r > 0.0 && vtri && dpos >= 0 &&
                          num<T>::abs(c.sV[dpos]) < A.stab_tol * vn;
        c.mi[MI_STAB] = stab ? 1 : 0;
        c.mi[MI_DPOS] = dpos;
        if (stab)
            c.mi[MI_FLAGS] = (c.mi[MI_FLAGS] | DIAF_FLAG_STABILIZED) & ~DIAF_FLAG_GAP_DEGENERATE;
        else if (dpos < 0 || num<T>::abs(c.sV[dpos]) < 1e-2 * vn)
            c.mi[MI_FLAGS] |= DIAF_FLAG_SMALL_DIAG;
    }
    __syncthreads();
    if (c.mi[MI_STAB]) {
        // v_jj = stab_r; on the other rows S of L the unit vector e^{i theta}
        // v1, v1 the top right singular vector of Mh = the columns of
        // M = L^{-1} B_L^* (the columns of Q^* up to a unitary factor) at S,
        // theta the argument of u1^* p (p the column at row j); w the
        // least-squares solution L^{-*} (M v) = L^{-*} (r p + e^{i theta} s1 u1).
        const int dpos = c.mi[MI_DPOS];
        const int ls = l - 1;
        for (int idx = tid; idx < k * l; idx += c.nt) {
            const int a = idx / l, t = idx % l;
            const int src = t < ls ? (t < dpos ? t : t + 1) : dpos;  // p goes last
            c.sX[a * c.xld + t] = num<T>::conj(bget(c, c.sL[src], a));
        }
        __syncthreads();
        lsolve(c, G, k, c.sX, l);
        if (ls > 0) jacobi_onesided(c, c.sX, k, ls, c.sVM);
        for (int t = tid; t < ls; t += c.nt) {
            double s2 = 0;
            for (int a = 0; a < k; ++a) s2 += num<T>::abs2(c.sX[a * c.xld + t]);
            c.sSig[t] = sqrt(s2);
        }
        __syncthreads();
        if (tid == 0) {
            int best = 0;
            T e = num<T>::one();
            if (ls > 0) {
                for (int t = 1; t < ls; ++t) if (c.sSig[t] > c.sSig[best]) best = t;
                const double s1 = c.sSig[best];
                double s2 = 0;
                for (int t = 0; t < ls; ++t) if (t != best && c.sSig[t] > s2) s2 = c.sSig[t];
                if (ls >= 2 && (!(s1 > 0) || (s1 * s1 - s2 * s2) / (s1 * s1) < 1e-6))
                    c.mi[MI_FLAGS] |= DIAF_FLAG_GAP_DEGENERATE;
                T z = num<T>::zero();
                for (int a = 0; a < k; ++a)
                    z += num<T>::conj(c.sX[a * c.xld + best]) * c.sX[a * c.xld + ls];
                const double az = num<T>::abs(z);
                if (az > 0.0) e = num<T>::div(z, az);
            }
            c.mi[MI_BEST] = best;
            c.md[MD_ERE] = num<T>::re(e);
            c.md[MD_EIM] = num<T>::im(e);
            c.sV[dpos] = num<T>::mk(A.stab_r);
            for (int t = 0; t < ls; ++t)
                c.sV[t < dpos ? t : t + 1] = e * c.sVM[t * ls + best];
        }
        __syncthreads();
        {
            const int best = c.mi[MI_BEST];
            T e;
            if constexpr (num<T>::is_complex) e = T{c.md[MD_ERE], c.md[MD_EIM]};
            else e = c.md[MD_ERE];
            for (int a = tid; a < k; a += c.nt) {
                T u = num<T>::mk(A.stab_r) * c.sX[a * c.xld + ls];
                if (ls > 0) u += e * c.sX[a * c.xld + best];
                c.sX[a * c.xld + l] = u;
            }
        }
        __syncthreads();
        for (int a = tid; a < k; a += c.nt) c.sX[a * c.xld] = c.sX[a * c.xld + l];
        __syncthreads();
        lhsolve(c, G, k, c.sX, 1);
        for (int a = tid; a < k; a += c.nt) c.sW[a] = c.sX[a * c.xld];
        __syncthreads();
    }
    bmul(c, m, c.sW, c.sY);
    if (tid == 0)
        for (int t = 0; t < l; ++t) c.sY[c.sL[t]] -= c.sV[t];
    __syncthreads();
    double s = 0;
    if (tid < 64)
        for (int i = tid; i < m; i += 64) s += num<T>::abs2(c.sY[i]);
    double r2 = wave0_sum(c, s);
    // unit-norm w: B without the rows of L has fewer rows than columns, or
    // its smallest singular value (here the residual) is negligible against
    // its Frobenius norm
    if (tid == 0 && A.mode == 1 && (m - l < k || r2 <= 1e-14 * c.md[MD_FRO2]))
        c.mi[MI_FLAGS] |= DIAF_FLAG_RANK_DEFICIENT;
    for (int a = tid; a < k; a += c.nt) A.Wval[jb + a] = c.sW[a];
    if (tid == 0) {
        // V column sorted by row (local order = global order)
        for (int a = 1; a < l; ++a) {
            int key = c.sL[a];
            T vv = c.sV[a];
            int b = a - 1;
            while (b >= 0 && c.sL[b] > key) { c.sL[b + 1] = c.sL[b]; c.sV[b + 1] = c.sV[b]; --b; }
            c.sL[b + 1] = key;
            c.sV[b + 1] = vv;
        }
        for (int t = 0; t < lmax; ++t) {
            A.Vrows[(size_t)j * lmax + t] = t < l ? c.sR[c.sL[t]] : -1;
            A.Vvals[(size_t)j * lmax + t] = t < l ? c.sV[t] : num<T>::zero();
        }
        A.rcol[j] = sqrt(r2);
        A.bnorm[j] = sqrt(c.md[MD_BN2]);
        A.flags[j] = (uint32_t)c.mi[MI_FLAGS];
        A.lcount[j] = l;
    }
    __syncthreads();
}

template <class T, bool IN_LDS>
__global__ void __launch_bounds__(GNT, 4) factor_generic_kernel(FactorArgs<T> A, int kcap, int tcap,
                                                             int tcap2, int lcap, int nmats_here,
                                                             unsigned char* gws, size_t slot_bytes,
                                                             T* gmats, size_t lds_split)
{
    extern __shared__ __align__(16) unsigned char lds_dyn[];
    unsigned char* base = IN_LDS ? lds_dyn : gws + (size_t)blockIdx.x * slot_bytes;
    const GenLayout Lo =
        gen_layout(kcap, tcap, tcap2, lcap, sizeof(T), nmats_here, IN_LDS ? 0 : lds_split);
    // the array's address: LDS or the block's global slot
    const auto at = [&](int id, size_t off) -> unsigned char* {
        return ((Lo.in_lds >> id) & 1u) ? lds_dyn + off : base + off;
    };
    GenCtx<T> c;
    c.tid = threadIdx.x;
    c.nt = blockDim.x;
    // the arrays placed first (flag and reduction slots, J_j and its column
    // offsets, the V rows and picks, w) always lie in LDS for kcap, lcap <=
    // 256; typed as LDS here so their reads are LDS reads, not flat ones
    c.sJ = (int32_t*)(lds_dyn + Lo.oJ);
    c.sOff = (int32_t*)(lds_dyn + Lo.oOff);
    c.sKey = (uint64_t*)at(GA_KEY, Lo.oKey);
    c.sScore = (double*)at(GA_KEY, Lo.oKey);
    c.sVal = (T*)at(GA_VAL, Lo.oVal);
    c.sLrow = (uint16_t*)at(GA_LROW, Lo.oLrow);
    c.sCol = (uint16_t*)at(GA_COL, Lo.oCol);
    c.sPos = (uint16_t*)at(GA_POS, Lo.oPos);
    c.sRowptr = (uint16_t*)at(GA_ROWPTR, Lo.oRowptr);
    c.sR = (int32_t*)at(GA_R, Lo.oR);
    c.sRank = (int32_t*)at(GA_RANK, Lo.oRank);
    c.sY = (T*)at(GA_Y, Lo.oY);
    c.sW = (T*)(lds_dyn + Lo.oW);
    c.sX = (T*)at(GA_X, Lo.oX);
    c.sVM = (T*)at(GA_VM, Lo.oVM);
    c.sSig = (double*)at(GA_SIG, Lo.oSig);
    c.sV = (T*)at(GA_V, Lo.oV);
    c.sL = (int32_t*)(lds_dyn + Lo.oL);
    c.sSel = (int32_t*)(lds_dyn + Lo.oSel);
    c.sRed = (double*)(lds_dyn + Lo.oRed);
    c.mi = (int*)(lds_dyn + Lo.oMisc);
    c.md = (double*)(lds_dyn + Lo.oMisc);
    c.xld = lcap + 1;
    const size_t kk = (size_t)kcap * kcap;
    // global k x k matrices (when not here): 1 per block for unit-norm v, 3 otherwise
    T* mats = nmats_here ? (T*)(base + Lo.oMats)
                         : gmats + (size_t)blockIdx.x * (A.mode == 0 ? 1 : 3) * kk;
    c.G = mats;
    c.E = mats + kk;
    c.Z = mats + 2 * kk;
    for (int q = blockIdx.x; q < A.ncols; q += gridDim.x) factor_one_column(A, A.cols[q], c);
}

template <class T>
size_t generic_lds_bytes(int kcap, int tcap, int lcap, int with_mats)
{
    int tcap2 = 1;
    while (tcap2 < tcap) tcap2 <<= 1;
    return gen_layout(kcap, tcap, tcap2, lcap, sizeof(T), with_mats).total;
}

// Placement of a size class: working set in LDS (with or without the k x k
// matrices) when it fits, otherwise a per-block slot of global memory.
// Columns of at most 32 unknowns run one wave per workgroup.
struct GenPlan {
    bool in_lds;
    bool mats_here;
    int nmats;          // k x k matrices per column: 1 (unit-norm v) or 3
    int nt;             // threads per workgroup
    size_t lds_bytes;   // dynamic LDS
    size_t slot_bytes;  // global slot per block (in_lds == false)
    bool need_gmats;    // separate global k x k matrices
    size_t lds_split;   // in_lds == false: LDS budget of the split layout (0: none)
};

// LDS budget of the split layout (in_lds == false): with the kernel's 8 KB
// of static LDS, four workgroups per CU
static constexpr size_t kGenSplitLds = 32 * 1024;
// the arrays taken first (misc, reduction, offsets, J, L, picks, w) always
// fit in the LDS part for kcap, lcap <= 256 (checked at launch)
static_assert(kGenSplitLds >= sizeof(double) * (32 + GNT) + sizeof(int32_t) * (kGenMaxK + 1) +
                                  sizeof(int32_t) * 3 * kGenMaxK + 2 * sizeof(double) * kGenMaxK +
                                  7 * 16,
              "split LDS too small");

template <class T>
GenPlan generic_plan(int kcap, int tcap, int lcap, int mode, int nt_override = 0)
{
    GenPlan P{};
    P.nmats = mode == 0 ? 1 : 3;
    P.nt = kcap <= 32 ? 64 : 256;
    if (nt_override == 64 || nt_override == 128 || nt_override == 256 || nt_override == GNT)
        P.nt = nt_override;
    size_t with = generic_lds_bytes<T>(kcap, tcap, lcap, P.nmats);
    size_t without = generic_lds_bytes<T>(kcap, tcap, lcap, 0);
    if (with <= 64 * 1024) {
        P.in_lds = true; P.mats_here = true; P.lds_bytes = with;
    } else if (without <= 96 * 1024) {
        P.in_lds = true; P.mats_here = false; P.lds_bytes = without; P.need_gmats = true;
    } else {
        // slot in global memory, with the hot small arrays in LDS
        int tcap2 = 1;
        while (tcap2 < tcap) tcap2 <<= 1;
        const GenLayout L = gen_layout(kcap, tcap, tcap2, lcap, sizeof(T), P.nmats, kGenSplitLds);
        P.in_lds = false;
        P.mats_here = true;
        P.lds_split = kGenSplitLds;
        P.lds_bytes = L.total_lds;
        P.slot_bytes = (L.total + 255) & ~size_t(255);
    }
    return P;
}

template <class T>
size_t generic_global_bytes(int kcap, int tcap, int lcap, int mode, int nslots)
{
    GenPlan P = generic_plan<T>(kcap, tcap, lcap, mode);
    if (P.in_lds && !P.need_gmats) return 0;
    if (P.need_gmats) return sizeof(T) * P.nmats * (size_t)kcap * kcap * nslots;
    return P.slot_bytes * nslots;
}

template <class T>
Err launch_factor_generic(const FactorArgs<T>& A, int kcap, int tcap, int lcap, void* gws,
                          int nslots, FactorTune tune, hipStream_t st)
{
    if (A.ncols == 0) return {};
    if (tcap > 65535) return {DIAF_EUNSUPPORTED, "column too large"};
    if (kcap > kGenMaxK || lcap > kGenMaxK)
        return {DIAF_EUNSUPPORTED, "generic kernel: more than 256 W or V entries in a column"};
    int tcap2 = 1;
    while (tcap2 < tcap) tcap2 <<= 1;
    GenPlan P = generic_plan<T>(kcap, tcap, lcap, A.mode, tune.generic_nt);
    int grid = A.ncols;
    if (!(P.in_lds && !P.need_gmats)) {
        if (!gws) return {DIAF_EINVAL, "generic factor: workspace missing"};
        if (grid > nslots) grid = nslots;
    }
    if (grid > 65535 * 8) grid = 65535 * 8;
    if (P.in_lds) {
        auto kern = factor_generic_kernel<T, true>;
        DIAF_HIP_TRY(hipFuncSetAttribute((const void*)kern,
                                         hipFuncAttributeMaxDynamicSharedMemorySize,
                                         (int)P.lds_bytes));
        hipLaunchKernelGGL(kern, dim3(grid), dim3(P.nt), P.lds_bytes, st, A, kcap, tcap, tcap2,
                           lcap, P.mats_here ? P.nmats : 0, (unsigned char*)nullptr, (size_t)0,
                           (T*)gws, (size_t)0);
    } else {
        auto kern = factor_generic_kernel<T, false>;
        DIAF_HIP_TRY(hipFuncSetAttribute((const void*)kern,
                                         hipFuncAttributeMaxDynamicSharedMemorySize,
                                         (int)P.lds_bytes));
        hipLaunchKernelGGL(kern, dim3(grid), dim3(P.nt), P.lds_bytes, st, A, kcap, tcap, tcap2,
                           lcap, P.nmats, (unsigned char*)gws, P.slot_bytes, (T*)nullptr,
                           P.lds_split);
    }
    DIAF_HIP_TRY(hipGetLastError());
    return {};
}

template <class T>
double generic_occupancy(int kcap, int tcap, int lcap, int mode, FactorTune tune)
{
    GenPlan P = generic_plan<T>(kcap, tcap, lcap, mode, tune.generic_nt);
    int nb = 0;
    const void* k = P.in_lds ? (const void*)factor_generic_kernel<T, true>
                             : (const void*)factor_generic_kernel<T, false>;
    if (P.in_lds &&
        hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)P.lds_bytes) !=
            hipSuccess)
        return 0.0;
    if (!P.in_lds &&
        hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)P.lds_bytes) !=
            hipSuccess)
        return 0.0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, P.nt, P.lds_bytes) != hipSuccess)
        return 0.0;
    return nb * (P.nt / 64) / 4.0;
}

template double generic_occupancy<double>(int, int, int, int, FactorTune);
template double generic_occupancy<zc>(int, int, int, int, FactorTune);

template Err launch_factor_generic<double>(const FactorArgs<double>&, int, int, int, void*, int,
                                           FactorTune, hipStream_t);
template Err launch_factor_generic<zc>(const FactorArgs<zc>&, int, int, int, void*, int, FactorTune,
                                       hipStream_t);
template size_t generic_global_bytes<double>(int, int, int, int, int);
template size_t generic_global_bytes<zc>(int, int, int, int, int);

}  // namespace diaf
