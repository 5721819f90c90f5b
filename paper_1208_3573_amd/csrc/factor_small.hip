// Small-column kernel for both basic algorithms (unit-norm columns of V,
// paper Section 2.1, or of W, Section 2.2): one wave per column, |J_j| <= 32, shadow |R_j| <= 64,
// at most 256 gathered entries and |L_j| <= 8.  Columns outside these limits,
// and unit-norm-w columns whose block without the V rows is rank deficient,
// are appended to a deferred list for the generic kernel.
//
// Per column, with B = A(R_j, J_j) and G = B^* B:
//   * shadow R_j: the gathered row indices are deduplicated in an LDS hash
//     table and the <= 64 distinct rows sorted across the wave with a
//     register bitonic network; row-ordered access (CSR) is built with
//     per-row counts, a wave scan and a per-row sort;
//   * G: the rows of every column of B form a 64-bit mask over the shadow, so
//     each entry G(a, b) visits only the rows common to columns a and b (in
//     ascending row order); the packed upper triangle goes to LDS;
//   * G^{-1} by the symmetric sweep (Gauss-Jordan), lane c holding column c
//     in registers and the pivot row broadcast through LDS; all later solves
//     are products of G^{-1} with dense k-vectors:
//   * seed w0 = G^{-1} b_j^* (V_0 = diagonals, Example 2.1), scores
//     |(B w0)_i| on the admissible rows and the top-(l-1) selection with the
//     1e-10 tie band (Section 3.1);
//   * Y = G^{-1} B_L^*, H = B_L Y (l x l) = M^* M for the paper's M_j
//     (eq. 2.3).  H is positive semidefinite with eigenvalues in [0, 1], so
//     its top eigenvector is the limit of the trace-normalised powers
//     H^(2^s): repeated squaring, one lane per entry of the padded 8 x 8
//     matrix, until the normalised power is rank one to 1e-12 (the angle
//     error then falls below 1e-24 after one more squaring); w = Y v
//     (eq. 2.4);
//   * phase (diagonal of V real positive), residual ||B w - v|| in FP64.
#include "dcommon.h"
#include "factor_kernels.h"

namespace diaf {

static constexpr int SKM = 32;   // max |J_j|
static constexpr int SMM = 64;   // max shadow size
static constexpr int STM = 256;  // max gathered entries
static constexpr int SLM = 8;    // max |L_j|
static constexpr int SHS = 256;  // hash slots

static constexpr int STRI = SKM * (SKM + 1) / 2;  // packed upper triangle of G

static constexpr int PMS = SKM + 1;  // column stride of Pm (odd: no bank conflicts)

// Packed upper-triangle index of G(a, b), a <= b (column b holds rows 0..b).
__device__ inline int tri(int a, int b) { return b * (b + 1) / 2 + a; }

template <class T, int MODE>
struct SmallLds {
    T eval[STM];  // gathered values, column by column in J order
    T Gk[MODE == 1 ? STRI : 1];  // unit-norm w: packed G, kept for two solves
    union {
        struct {  // gather and shadow
            int hkey[SHS];   // hash of the shadow rows
            union {
                int tmp[SMM];
                int rcnt[SMM];
            };
            uint8_t eslot[STM];
            uint8_t hval[SHS];
        } sh;
        struct {  // Gram matrix (until the sweep)
            T Gt[STRI];            // packed upper triangle of G
            uint64_t cmask[SKM];   // rows (local ids) of each column of B
        } gr;
        T bc[2][SKM];  // pivot row of the sweep (double-buffered)
        T Pm[MODE == 1 ? SKM * PMS : 1];  // unit-norm w: power being squared
        struct {
            union {
                T U[SLM * SKM];  // U[t][i] = conj(B(L_t, i)), dense k-vectors
                struct {
                    T P[SLM * SLM];   // power of H being squared (after Y)
                    T v[SLM];
                    T Hs[SLM * SLM];  // H itself, for the constrained solve
                    T vs[SLM];        // its top eigenvector on the rows S
                };
            };
            T Y[SKM * SLM];  // Y[i][t] = (G^{-1} U)(i, t)
            T w[SKM];
        } post;
    };
    int a0[SKM];  // start of each column of B in A
    int off[SKM + 1];
    int R[SMM];  // shadow rows, ascending
    int rptr[SMM + 1];
    int L[SLM];
    uint8_t eloc[STM];
    uint8_t ecol[STM];
    uint8_t csr[STM];
};

// v of lane src (the same src on every lane) on every lane, by readlane
template <class T>
__device__ inline T bcast(T v, int src)
{
    if constexpr (num<T>::is_complex) return T{readlane_f64(v.x, src), readlane_f64(v.y, src)};
    else return readlane_f64(v, src);
}

// Value of lane ^ 32 (the other half of the wave).
template <class T>
__device__ inline T shfl_xor32(T v)
{
    if constexpr (num<T>::is_complex) return T{xor32_f64(v.x), xor32_f64(v.y)};
    else return xor32_f64(v);
}

// Whole-wave scan and reductions (every lane active): DPP and readlane,
// no LDS round trips.
__device__ inline int wave_incl_scan(int x, int) { return dpp_wave_incl_scan(x); }
__device__ inline double wave_sum(double x) { return dpp_wave_sum(x); }
__device__ inline double wave_max(double x) { return dpp_wave_max(x); }

// 1 / d from the hardware reciprocal and two Newton steps, r <- r + r (1 - d r)
// (each step squares the relative error; the result is within an ulp or
// so of the correctly rounded quotient), 5 instructions against 13 for
// the IEEE division.  Callers guard d away from zero.
__device__ __forceinline__ double recip_nr(double d)
{
    double r = __builtin_amdgcn_rcp(d);
    r = __builtin_fma(r, __builtin_fma(-d, r, 1.0), r);
    return __builtin_fma(r, __builtin_fma(-d, r, 1.0), r);
}

// Symmetric sweep (Gauss-Jordan) of a Hermitian k x k matrix padded with
// the identity to 32 x 32.  Lanes c and c + 32 hold rows 0..15 and 16..31 of
// column c in g (hf = lane / 32).  Step p: a_qc -= a_qp a_pc / d (c != p),
// the pivot column becomes a_qp / d and entry p of every column a_pc / d
// (-1/d on the pivot); the result is minus the inverse.  The iterate stays
// Hermitian, so a_qp = conj(a_pq): the half holding row p publishes a_pc for
// every column and all lanes read the pivot row back from LDS.  Register
// indices are static.
template <class T>
__device__ __forceinline__ void sweep_inverse(T (&g)[SKM / 2], int k, int c, int hf, double maxd,
                                              T (*bc)[SKM], uint32_t& flags)
{
    constexpr int SKH = SKM / 2;
#pragma unroll
    for (int p = 0; p < SKM; ++p) {
        if (p < k) {
            T* b = bc[p & 1];
            if ((p / SKH) == hf) b[c] = g[p % SKH];
            __syncthreads();
            const double d = num<T>::re(b[p]);
            const bool zero = !(d > 1e-30 * maxd) || !isfinite(d);
            if (!(d > 1e-14 * maxd)) flags |= DIAF_FLAG_RANK_DEFICIENT;
            const double inv = zero ? 0.0 : recip_nr(d);
            const bool piv = (c == p);
            const T apc = b[c];
            const T coef = piv ? num<T>::mk(1.0 - inv) : apc * inv;
            const T* brow = b + hf * SKH;
#pragma unroll
            for (int i = 0; i < SKH; ++i) g[i] -= num<T>::conj(brow[i]) * coef;
            if ((p / SKH) == hf) g[p % SKH] = piv ? num<T>::mk(zero ? 0.0 : -inv) : apc * inv;
        }
    }
    __syncthreads();
}

// Top eigenvector of the Hermitian positive semidefinite l x l matrix (l <=
// 8) whose entry (hs, ht) lane hs * 8 + ht holds in h (zero outside l x l),
// by repeated squaring: P = H / tr(H), then P <- P^2 / tr(P^2), with
// tr(P^2) = ||P||_F^2.  For P = sum mu_i v_i v_i^* (sum mu_i = 1),
// 1 - tr(P^2) ~ 2 mu_2, so the loop stops one squaring after
// 1 - tr(P^2) < 1e-12.  The eigenvector is the column of the last power
// with the largest diagonal entry (lowest index on ties), normalised, into
// out[0..l).  Returns false when the trace is not positive or 25 squarings
// did not reach rank one (the top eigenvalue is then separated from the
// next by less than a relative 1e-6).  P is LDS scratch of 64 entries.
template <class T>
__device__ __forceinline__ bool top_eig_h(T h, int l, int hs, int ht, int lane, T* P, T* out)
{
    const double tr = wave_sum((hs == ht) ? num<T>::re(h) : 0.0);
    bool conv = false, ok = true;
    if (!(tr > 0.0) || !isfinite(tr)) {
        h = (hs == 0 && ht == 0) ? num<T>::one() : num<T>::zero();
        ok = false;
        conv = true;
    } else {
        h = num<T>::div(h, tr);
    }
    for (int s = 0; s < 25 && !conv; ++s) {
        const double f = wave_sum(num<T>::abs2(h));
        conv = (1.0 - f) < 1e-12;
        P[lane] = h;
        __syncthreads();
        T acc = num<T>::zero();
#pragma unroll
        for (int q = 0; q < SLM; ++q) acc += P[hs * SLM + q] * P[q * SLM + ht];
        __syncthreads();
        h = num<T>::div(acc, f);
    }
    if (!conv) ok = false;
    const double dg = (hs == ht && hs < l) ? num<T>::re(h) : -1.0;
    const double dmx = wave_max(dg);
    const uint64_t cm = __ballot(hs == ht && hs < l && dg == dmx);
    const int cstar = (__ffsll((unsigned long long)cm) - 1) >> 3;
    if (ht == cstar && hs < SLM) out[hs] = h;
    __syncthreads();
    double nv = 0.0;
    for (int t = 0; t < l; ++t) nv += num<T>::abs2(out[t]);
    nv = sqrt(nv);
    __syncthreads();
    if (lane < l) out[lane] = num<T>::div(out[lane], nv);
    __syncthreads();
    return ok;
}

// Top eigenvector of a Hermitian positive semidefinite k x k matrix P held
// as half-columns (as in sweep_inverse) and zero outside k x k: the
// trace-normalised powers P^(2^s) by repeated squaring until the power is
// rank one to 1e-12 (one more squaring after that), then the column with
// the largest diagonal entry (lowest index on ties), normalised, into out.
// Returns false if 25 squarings did not reach rank one (the top eigenvalue
// is then separated from the next by less than a relative 1e-6).
template <class T>
__device__ __forceinline__ bool top_eig_k(T (&pv)[SKM / 2], int k, int c, int hf, int lane, T* Pm,
                                          T* out)
{
    constexpr int SKH = SKM / 2;
    double dsum = 0.0;
#pragma unroll
    for (int i = 0; i < SKH; ++i)
        if (hf * SKH + i == c && c < k) dsum += num<T>::re(pv[i]);
    const double tr = wave_sum(dsum);
    bool conv = false;
    if (!(tr > 0.0) || !isfinite(tr)) {
#pragma unroll
        for (int i = 0; i < SKH; ++i)
            pv[i] = (hf * SKH + i == c && c == 0) ? num<T>::one() : num<T>::zero();
        conv = true;
    } else {
#pragma unroll
        for (int i = 0; i < SKH; ++i) pv[i] = num<T>::div(pv[i], tr);
    }
    const bool ok = conv ? false : true;
    for (int s = 0; s < 25 && !conv; ++s) {
        double fs = 0.0;
#pragma unroll
        for (int i = 0; i < SKH; ++i) fs += num<T>::abs2(pv[i]);
        const double f = wave_sum(fs);
        conv = (1.0 - f) < 1e-12;
#pragma unroll
        for (int i = 0; i < SKH; ++i) Pm[c * PMS + hf * SKH + i] = pv[i];
        __syncthreads();
        // (P^2)(r, c) = sum_q conj(P(q, r)) P(q, c): q outer (entries beyond
        // k are zero), the rows r of this lane's half in registers
        T acc[SKH];
#pragma unroll
        for (int i = 0; i < SKH; ++i) acc[i] = num<T>::zero();
        for (int q = 0; q < k; ++q) {
            const T pqc = Pm[c * PMS + q];
#pragma unroll
            for (int i = 0; i < SKH; ++i)
                acc[i] += num<T>::conj(Pm[(hf * SKH + i) * PMS + q]) * pqc;
        }
#pragma unroll
        for (int i = 0; i < SKH; ++i) pv[i] = num<T>::div(acc[i], f);
        __syncthreads();
    }
    double dg = -1.0;
#pragma unroll
    for (int i = 0; i < SKH; ++i)
        if (hf * SKH + i == c && c < k) dg = num<T>::re(pv[i]);
    const double dmx = wave_max(dg);
    const uint64_t cm = __ballot(dg == dmx && dg >= 0.0);
    const int cstar = (__ffsll((unsigned long long)cm) - 1) & (SKM - 1);
    if (c == cstar) {
#pragma unroll
        for (int i = 0; i < SKH; ++i)
            if (hf * SKH + i < k) out[hf * SKH + i] = pv[i];
    }
    __syncthreads();
    const double nv = sqrt(wave_sum(lane < k ? num<T>::abs2(out[lane]) : 0.0));
    __syncthreads();
    if (lane < k) out[lane] = num<T>::div(out[lane], nv);
    __syncthreads();
    return ok && conv;
}

// Unit-norm w: loads G - sum_{t<nt} U_t U_t^* + shift * I (the Gram matrix
// of B without the rows held in U) as half-columns, inverts it by the
// sweep and takes the top eigenvector of the inverse, i.e. the bottom
// eigenvector of the downdated Gram matrix, into out (unit norm).
template <class T, int MODE>
__device__ __forceinline__ bool bottom_eig_w(SmallLds<T, MODE>& S, int k, int nt, int c, int hf,
                                             int lane, double maxd, double shift, T* out)
{
    constexpr int SKH = SKM / 2;
    T g[SKH];
#pragma unroll
    for (int i = 0; i < SKH; ++i) {
        const int r = hf * SKH + i;
        if (r < k && c < k) {
            T a = r <= c ? S.Gk[tri(r, c)] : num<T>::conj(S.Gk[tri(c, r)]);
            for (int t = 0; t < nt; ++t)
                a -= S.post.U[t * SKM + r] * num<T>::conj(S.post.U[t * SKM + c]);
            if (r == c) a += num<T>::mk(shift);
            g[i] = a;
        } else {
            g[i] = (r == c) ? num<T>::one() : num<T>::zero();
        }
    }
    __syncthreads();  // U has been read; bc and Pm alias it
    uint32_t unused = 0;
    sweep_inverse(g, k, c, hf, maxd, S.bc, unused);
#pragma unroll
    for (int i = 0; i < SKH; ++i) {
        const int r = hf * SKH + i;
        g[i] = (r < k && c < k) ? -g[i] : num<T>::zero();
    }
    return top_eig_k(g, k, c, hf, lane, S.Pm, out);
}

template <class T, int MODE>
__device__ __forceinline__ void small_column(const FactorArgs<T>& A, int j, SmallLds<T, MODE>& S,
                                             int* deferred, int* ndeferred, DeferBuf& db)
{
    // opaque per call: keeps lane-derived addresses from being hoisted out of
    // the column loop (they would stay live in registers for the whole kernel)
    int lane = threadIdx.x;
    __asm__ volatile("" : "+v"(lane));
    const int jb = A.Jcp[j];
    const int k = A.Jcp[j + 1] - jb;
    const int lmax = A.lmax;
    // ---- 1. J_j and gather offsets ----
    int len = 0;
    if (lane < k && k <= SKM) {
        const int c = A.Jri[jb + lane];
        const int a0 = A.Acp[c];
        S.a0[lane] = a0;
        len = A.Acp[c + 1] - a0;
    }
    int inc = wave_incl_scan(len, lane);
    if (lane < k && k <= SKM) S.off[lane + 1] = inc;
    if (lane == 0) S.off[0] = 0;
    const int Tn = __builtin_amdgcn_readlane(inc, 63);
    for (int s = lane; s < SHS; s += 64) S.sh.hkey[s] = -1;
    __syncthreads();
    if (k > SKM || Tn > STM) {
        defer_push(db, j, lane, deferred, ndeferred);
        return;
    }
    // ---- 2. gather; shadow rows into the hash table ----
    // every load of this lane's entries (t = lane + 64 i) is issued before
    // the first is used; the rows new to the table are counted per round, so
    // a column whose shadow exceeds SMM rows is deferred without filling it
    constexpr int EPL = STM / 64;
    int grow[EPL];
    T gval[EPL];
#pragma unroll
    for (int i = 0; i < EPL; ++i) {
        const int t = lane + 64 * i;
        grow[i] = 0;
        gval[i] = num<T>::zero();
        if (t < Tn) {
            int lo = 0, hi = k - 1;
            while (lo < hi) {
                int mid = (lo + hi + 1) >> 1;
                if (S.off[mid] <= t) lo = mid; else hi = mid - 1;
            }
            const int p = S.a0[lo] + (t - S.off[lo]);
            grow[i] = A.Ari[p];
            gval[i] = A.Aval[p];
            S.ecol[t] = (uint8_t)lo;
        }
    }
    int mnew = 0;
#pragma unroll
    for (int i = 0; i < EPL; ++i) {
        const int t = lane + 64 * i;
        bool fresh = false;
        if (t < Tn) {
            const int row = grow[i];
            S.eval[t] = gval[i];
            unsigned h = ((unsigned)row * 2654435761u) >> 24;
            for (;;) {
                const int prev = atomicCAS(&S.sh.hkey[h], -1, row);
                if (prev == -1 || prev == row) { fresh = prev == -1; break; }
                h = (h + 1) & (SHS - 1);
            }
            S.sh.eslot[t] = (uint8_t)h;
        }
        mnew += __popcll(__ballot(fresh));
        if (mnew > SMM) break;
    }
    __syncthreads();
    if (mnew > SMM) {
        defer_push(db, j, lane, deferred, ndeferred);
        return;
    }
    // ---- 3. shadow: local row ids by ascending row ----
    int m = 0;
    for (int q = 0; q < SHS / 64; ++q) {
        int s = q * 64 + lane;
        int key = S.sh.hkey[s];
        bool occ = key != -1;
        uint64_t mask = __ballot(occ);
        int pos = m + __popcll(mask & ((1ull << lane) - 1ull));
        if (occ && pos < SMM) { S.R[pos] = key; S.sh.tmp[pos] = s; }
        m += __popcll(mask);
    }
    __syncthreads();
    if (m > SMM) {
        defer_push(db, j, lane, deferred, ndeferred);
        return;
    }
    int myrow = lane < m ? S.R[lane] : 0x7fffffff;
    int myslot = lane < m ? S.sh.tmp[lane] : 0;
    for (int kk = 2; kk <= 64; kk <<= 1) {
        for (int jj = kk >> 1; jj > 0; jj >>= 1) {
            int orow = __shfl_xor(myrow, jj);
            int oslot = __shfl_xor(myslot, jj);
            bool up = (lane & kk) == 0;
            bool lower = (lane & jj) == 0;
            bool take = (lower == up) ? (orow < myrow) : (orow > myrow);
            if (take) { myrow = orow; myslot = oslot; }
        }
    }
    __syncthreads();
    if (lane < m) {
        S.R[lane] = myrow;
        S.sh.hval[myslot] = (uint8_t)lane;
    }
    if (lane < SMM) S.sh.rcnt[lane] = 0;
    const uint64_t dmask = __ballot(lane < m && myrow == j);
    const int dj = dmask ? __ffsll((unsigned long long)dmask) - 1 : -1;
    __syncthreads();
    double bn2 = 0.0;
    for (int t = lane; t < Tn; t += 64) {
        int lr = S.sh.hval[S.sh.eslot[t]];
        S.eloc[t] = (uint8_t)lr;
        atomicAdd(&S.sh.rcnt[lr], 1);
        bn2 += num<T>::abs2(S.eval[t]);
    }
    bn2 = wave_sum(bn2);
    __syncthreads();
    {
        int rc = lane < m ? S.sh.rcnt[lane] : 0;
        int ri = wave_incl_scan(rc, lane);
        S.rptr[lane + 1] = ri;
        if (lane == 0) S.rptr[0] = 0;
        S.sh.rcnt[lane] = 0;
    }
    __syncthreads();
    for (int t = lane; t < Tn; t += 64) {
        int lr = S.eloc[t];
        int pos = S.rptr[lr] + atomicAdd(&S.sh.rcnt[lr], 1);
        S.csr[pos] = (uint8_t)t;
    }
    __syncthreads();
    if (lane < m) {  // ascending entry index = ascending column within each row
        int b = S.rptr[lane], e = S.rptr[lane + 1];
        for (int p = b + 1; p < e; ++p) {
            uint8_t key = S.csr[p];
            int q = p - 1;
            while (q >= b && S.csr[q] > key) { S.csr[q + 1] = S.csr[q]; --q; }
            S.csr[q + 1] = key;
        }
    }
    __syncthreads();
    if (dj < 0) {
        for (int a = lane; a < k; a += 64) A.Wval[jb + a] = num<T>::zero();
        for (int t = lane; t < lmax; t += 64) {
            A.Vrows[(size_t)j * lmax + t] = -1;
            A.Vvals[(size_t)j * lmax + t] = num<T>::zero();
        }
        if (lane == 0) {
            A.rcol[j] = 0.0;
            A.bnorm[j] = sqrt(bn2);
            A.flags[j] = DIAF_FLAG_NO_DIAG_ROW;
            A.lcount[j] = 0;
        }
        return;
    }
    uint32_t flags = 0;
    // ---- 4. Gram matrix: G(a, b) over the rows common to columns a and b ----
    // The diagonal G(a, a) comes from column a's own entries (ascending
    // rows, as the pair loop would take them); the strictly upper pairs
    // then loop only over their few common rows.
    if (lane < k) {
        uint64_t msk = 0;
        T dacc = num<T>::zero();
        for (int t = S.off[lane]; t < S.off[lane + 1]; ++t) {
            msk |= 1ull << S.eloc[t];
            dacc += num<T>::cmul(S.eval[t], S.eval[t]);
        }
        S.gr.cmask[lane] = msk;
        if constexpr (MODE == 1) S.Gk[tri(lane, lane)] = dacc;
        else S.gr.Gt[tri(lane, lane)] = dacc;
    }
    __syncthreads();
    const int npair = k * (k - 1) / 2;
    for (int q = lane; q < npair; q += 64) {
        // strictly upper pair q = bb (bb - 1) / 2 + aa, aa < bb
        int bb = (int)((sqrtf(8.0f * (float)q + 1.0f) + 1.0f) * 0.5f);
        while (bb * (bb - 1) / 2 > q) --bb;
        while ((bb + 1) * bb / 2 <= q) ++bb;
        const int aa = q - bb * (bb - 1) / 2;
        const uint64_t ma = S.gr.cmask[aa], mb = S.gr.cmask[bb];
        uint64_t common = ma & mb;
        const int oa = S.off[aa], ob = S.off[bb];
        T acc = num<T>::zero();
        while (common) {
            const int r = __ffsll((unsigned long long)common) - 1;
            const uint64_t below = (1ull << r) - 1ull;
            acc += num<T>::cmul(S.eval[oa + __popcll(ma & below)], S.eval[ob + __popcll(mb & below)]);
            common &= common - 1ull;
        }
        if constexpr (MODE == 1) S.Gk[tri(aa, bb)] = acc;
        else S.gr.Gt[tri(aa, bb)] = acc;
    }
    __syncthreads();
    // ---- 5. unit-norm v: G^{-1} by the symmetric sweep ----
    // Lanes c and c + 32 hold rows 0..15 and 16..31 of column c (hf = lane /
    // 32 picks the half); the sweep leaves -G^{-1} there.  Unit-norm w keeps
    // G packed in LDS and solves twice (seed and final) further down.
    const int c = lane & (SKM - 1), hf = lane >> 5;
    constexpr int SKH = SKM / 2;
    T g[SKH];
    const T* Gp = (MODE == 1) ? S.Gk : S.gr.Gt;
    double maxd = lane < k ? num<T>::re(Gp[tri(c, c)]) : 0.0;
    maxd = wave_max(maxd);
    // shift for unit-norm w: the downdated Gram matrix plus shift * I is
    // positive definite, and the shift leaves its eigenvectors unchanged
    const double shift = 1e-12 * maxd;
    if constexpr (MODE == 0) {
#pragma unroll
        for (int i = 0; i < SKH; ++i) {
            const int r = hf * SKH + i;
            if (r < k && c < k) g[i] = r <= c ? S.gr.Gt[tri(r, c)] : num<T>::conj(S.gr.Gt[tri(c, r)]);
            else g[i] = (r == c) ? num<T>::one() : num<T>::zero();
        }
        __syncthreads();  // Gt is dead from here on; bc and post alias it
        sweep_inverse(g, k, c, hf, maxd, S.bc, flags);
    }
    // ---- 6. V pattern ----
    const bool topk =
        A.vrule == V_TOPK_LOWER || A.vrule == V_TOPK_UPPER || A.vrule == V_TOPK_BLOCK;
    const bool lev = MODE == 0 && (A.vrule == V_LEV_LOWER || A.vrule == V_LEV_UPPER);
    const bool lowerrule = A.vrule == V_TOPK_LOWER || A.vrule == V_LEV_LOWER;
    int l = 0;
    if (topk || lev) {
      // admissible: the strict triangle, or the other rows of j's diagonal
      // block for a block diagonal V (Section 5)
      const bool adm =
          lane < m && (A.vrule == V_TOPK_BLOCK
                           ? (myrow != j && myrow >= A.vblk[2 * j] && myrow < A.vblk[2 * j + 1])
                           : (lowerrule ? myrow > j : myrow < j));
      double sc = -1.0;
      if (topk) {
        // w0 = G^{-1} u with u = conj(B(j, :)): lane c takes the product of
        // its column of -G^{-1} (Hermitian) with u
        if (lane < SKM) S.post.U[lane] = num<T>::zero();
        __syncthreads();
        {
            const int pb = S.rptr[dj], pe = S.rptr[dj + 1];
            if (lane < pe - pb) {
                const int t = S.csr[pb + lane];
                S.post.U[S.ecol[t]] = num<T>::conj(S.eval[t]);
            }
        }
        __syncthreads();
        if constexpr (MODE == 0) {
            T acc = num<T>::zero();
#pragma unroll
            for (int i = 0; i < SKH; ++i) acc -= num<T>::conj(g[i]) * S.post.U[hf * SKH + i];
            acc += shfl_xor32(acc);
            if (lane < k) S.post.w[lane] = acc;
        } else {
            // seed of the second basic algorithm: bottom eigenvector of
            // G - b_j^* b_j (B without row j)
            bottom_eig_w(S, k, 1, c, hf, lane, maxd, shift, S.post.w);
        }
        __syncthreads();
        T yr = num<T>::zero();
        if (lane < m)
            for (int pp = S.rptr[lane]; pp < S.rptr[lane + 1]; ++pp) {
                int t = S.csr[pp];
                yr += S.eval[t] * S.post.w[S.ecol[t]];
            }
        sc = adm ? num<T>::abs(yr) : -1.0;
      } else {
        if constexpr (MODE == 0) {
            // Section 3.1's rule: the score of an admissible row i is the norm
            // of its column of Q^*, sqrt(h_i) with h_i = b_i G^{-1} b_i^*.
            // Batches of up to SLM rows go through U (conj rows, dense) and
            // Y = G^{-1} U as for B_L^* below; the row's lane forms b_i y_i.
            double hlev = 0.0;
            uint64_t rem = __ballot(adm);
            while (rem) {
                uint64_t bmask = 0;
                int nb = 0;
                while (rem && nb < SLM) {
                    bmask |= rem & (~rem + 1ull);
                    rem &= rem - 1ull;
                    ++nb;
                }
                for (int q2 = lane; q2 < SLM * SKM; q2 += 64) S.post.U[q2] = num<T>::zero();
                __syncthreads();
                const bool inb = (bmask >> lane) & 1ull;
                const int slot = __popcll(bmask & ((1ull << lane) - 1ull));
                if (inb)
                    for (int pp = S.rptr[lane]; pp < S.rptr[lane + 1]; ++pp) {
                        const int e = S.csr[pp];
                        S.post.U[slot * SKM + S.ecol[e]] = num<T>::conj(S.eval[e]);
                    }
                __syncthreads();
                for (int t = 0; t < nb; ++t) {
                    T acc = num<T>::zero();
#pragma unroll
                    for (int i = 0; i < SKH; ++i)
                        acc -= num<T>::conj(g[i]) * S.post.U[t * SKM + hf * SKH + i];
                    acc += shfl_xor32(acc);
                    if (lane < k) S.post.Y[lane * SLM + t] = acc;
                }
                __syncthreads();
                if (inb) {
                    T h = num<T>::zero();
                    for (int pp = S.rptr[lane]; pp < S.rptr[lane + 1]; ++pp) {
                        const int e = S.csr[pp];
                        h += S.eval[e] * S.post.Y[S.ecol[e] * SLM + slot];
                    }
                    hlev = num<T>::re(h);
                }
                __syncthreads();
            }
            sc = adm ? sqrt(fmax(hlev, 0.0)) : -1.0;
        }
      }
        const uint64_t amask = __ballot(adm);
        const int nc = __popcll(amask);
        int lj = A.vcount < 1 ? 1 : A.vcount;
        if (lj > 1 + nc) lj = 1 + nc;
        if (MODE == 1) {  // keep B without the rows of L at least k rows tall
            const int cap = m - k > 1 ? m - k : 1;
            if (lj > cap) lj = cap;
        }
        if (lj > lmax) lj = lmax;
        const int q = lj - 1;
        __syncthreads();
        bool chosen = false;
        if (q > 0 && nc <= q) {
            chosen = adm;
        } else if (q > 0) {
            // the q-th largest score (ties: lower lane first), by q rounds of
            // extracting the maximum
            bool taken = false;
            double ss = 0.0;
            for (int r = 0; r < q; ++r) {
                const double cand = (adm && !taken) ? sc : -2.0;
                const double mx = wave_max(cand);
                const uint64_t bm = __ballot(adm && !taken && sc == mx);
                if (lane == __ffsll((unsigned long long)bm) - 1) taken = true;
                ss = mx;
            }
            const double hi = ss * (1.0 + 1e-10), lo = ss * (1.0 - 1e-10);
            const bool in = adm && sc > hi;
            const bool tie = adm && sc >= lo && sc <= hi;
            const uint64_t inmask = __ballot(in), tmask = __ballot(tie);
            const int need = q - __popcll(inmask);
            const int trank = __popcll(tmask & ((1ull << lane) - 1ull));
            chosen = in || (tie && trank < need);
            const bool edge = adm && ss > 0.0 &&
                              (fabs(sc - hi) <= 1e-12 * ss || fabs(sc - lo) <= 1e-12 * ss);
            if (__ballot(edge)) flags |= DIAF_FLAG_TIE_EDGE;
        }
        const uint64_t cmask = __ballot(chosen);
        if (chosen) S.L[1 + __popcll(cmask & ((1ull << lane) - 1ull))] = lane;
        if (lane == 0) S.L[0] = dj;
        l = 1 + __popcll(cmask);
    } else {
        int b = 0, e = 0;
        const int32_t* rows = nullptr;
        if (A.vrule == V_DIAG) {
            if (lane == 0) S.L[0] = dj;
            l = 1;
        } else {
            if (A.vrule == V_EXPLICIT) { b = A.Vcp_in[j]; e = A.Vcp_in[j + 1]; rows = A.Vri_in; }
            else { b = A.Acp[j]; e = A.Acp[j + 1]; rows = A.Ari; }
            for (int p0 = b; p0 < e; p0 += 64) {
                int lr = -1;
                int p = p0 + lane;
                if (p < e) {
                    int gi = rows[p];
                    bool keep = A.vrule == V_EXPLICIT || gi == j ||
                                (A.vrule == V_GS_UPPER ? gi < j : gi > j);
                    if (keep) {  // local id = position in the sorted shadow
                        int lo = 0, hi = m - 1;
                        while (lo <= hi) {
                            const int mid = (lo + hi) >> 1;
                            const int rv = S.R[mid];
                            if (rv == gi) { lr = mid; break; }
                            if (rv < gi) lo = mid + 1;
                            else hi = mid - 1;
                        }
                    }
                }
                uint64_t km = __ballot(lr >= 0);
                int pos = l + __popcll(km & ((1ull << lane) - 1ull));
                if (lr >= 0 && pos < SLM) S.L[pos] = lr;
                l += __popcll(km);
            }
            if (l > SLM || l > lmax) {
                __syncthreads();
                defer_push(db, j, lane, deferred, ndeferred);
                return;
            }
        }
    }
    __syncthreads();
    // ---- 7. Y = G^{-1} B_L^*, H = B_L Y ----
    for (int q = lane; q < SLM * SKM; q += 64) S.post.U[q] = num<T>::zero();
    __syncthreads();
    for (int t = 0; t < l; ++t) {
        const int r = S.L[t];
        const int pb = S.rptr[r], pe = S.rptr[r + 1];
        if (lane < pe - pb) {
            const int e = S.csr[pb + lane];
            S.post.U[t * SKM + S.ecol[e]] = num<T>::conj(S.eval[e]);
        }
    }
    __syncthreads();
    if constexpr (MODE == 0) {
        for (int t = 0; t < l; ++t) {
            T acc = num<T>::zero();
#pragma unroll
            for (int i = 0; i < SKH; ++i) acc -= num<T>::conj(g[i]) * S.post.U[t * SKM + hf * SKH + i];
            acc += shfl_xor32(acc);
            if (lane < k) S.post.Y[lane * SLM + t] = acc;
        }
        __syncthreads();
        const int hs = lane >> 3, ht = lane & 7;
        T h = num<T>::zero();
        if (hs < l && ht < l) {
            const int r = S.L[hs];
            for (int pp = S.rptr[r]; pp < S.rptr[r + 1]; ++pp) {
                int e = S.csr[pp];
                h += S.eval[e] * S.post.Y[S.ecol[e] * SLM + ht];
            }
        }
        // ---- 8. top eigenvector of H ----
        S.post.Hs[lane] = h;
        if (!top_eig_h(h, l, hs, ht, lane, S.post.P, S.post.v)) flags |= DIAF_FLAG_GAP_DEGENERATE;
        // w = Y v
        if (lane < k) {
            T acc = num<T>::zero();
            for (int t = 0; t < l; ++t) acc += S.post.Y[lane * SLM + t] * S.post.v[t];
            S.post.w[lane] = acc;
        }
        __syncthreads();
    } else {
        // final solve of the second basic algorithm (Section 2.2): w = bottom
        // eigenvector of G - B_L^* B_L (B without the rows of L), v = (B w)|_L
        if (!bottom_eig_w(S, k, l, c, hf, lane, maxd, shift, S.post.w))
            flags |= DIAF_FLAG_GAP_DEGENERATE;
        if (lane < l) {
            const int r = S.L[lane];
            T acc = num<T>::zero();
            for (int pp = S.rptr[r]; pp < S.rptr[r + 1]; ++pp) {
                const int e = S.csr[pp];
                acc += S.eval[e] * S.post.w[S.ecol[e]];
            }
            S.post.v[lane] = acc;
        }
        __syncthreads();
    }
    // ---- 9. phase ; residual ----
    T vt = lane < l ? S.post.v[lane] : num<T>::zero();
    const double vn = sqrt(wave_sum(lane < l ? num<T>::abs2(vt) : 0.0));
    const uint64_t dposm = __ballot(lane < l && S.L[lane] == dj);
    const int dpos = dposm ? __ffsll((unsigned long long)dposm) - 1 : -1;
    int piv;
    if (dpos >= 0 && num<T>::abs(bcast(vt, dpos)) >= 1e-8 * vn) {
        piv = dpos;
    } else {
        const double av = lane < l ? num<T>::abs(vt) : -1.0;
        const double mx = wave_max(av);
        // lowest global row among the maxima = lowest local row
        const int lr = lane < l ? S.L[lane] : 0x7fffffff;
        int cand = (lane < l && av == mx) ? lr : 0x7fffffff;
        cand = dpp_wave_min(cand);
        const uint64_t pm = __ballot(lane < l && av == mx && lr == cand);
        piv = __ffsll((unsigned long long)pm) - 1;
    }
    const T pvv = bcast(vt, piv);
    const T ph = num<T>::iszero(pvv) ? num<T>::one() : unit_conj_phase(pvv);
    vt = ph * vt;
    if (dpos < 0 || num<T>::abs(bcast(vt, dpos < 0 ? 0 : dpos)) < 1e-2 * vn)
        flags |= DIAF_FLAG_SMALL_DIAG;
    if (lane < l) S.post.v[lane] = vt;
    if (lane < k) S.post.w[lane] = ph * S.post.w[lane];
    __syncthreads();
    if constexpr (MODE == 0) {
        // Section 3.2: with a triangular V and |v_jj| < stab_tol ||v||, fix
        // v_jj = stab_r; on the other rows S of L put e^{i theta} vs, vs the
        // top eigenvector of H(S, S) (= the top right singular vector of the
        // columns of Q^* at S) and theta the argument of vs^* H(S, j) (the
        // first component of U^* p in the paper's notation); w = Y v, the
        // least-squares solution for that v (eq. 2.4).
        const bool vtri = A.vrule == V_DIAG || A.vrule == V_GS_UPPER || A.vrule == V_GS_LOWER ||
                          A.vrule == V_TOPK_UPPER || A.vrule == V_TOPK_LOWER ||
                          A.vrule == V_LEV_UPPER || A.vrule == V_LEV_LOWER;
        if (A.stab_r > 0.0 && vtri && dpos >= 0 && num<T>::abs(bcast(vt, dpos)) < A.stab_tol * vn) {
            flags = (flags | DIAF_FLAG_STABILIZED) & ~(DIAF_FLAG_SMALL_DIAG | DIAF_FLAG_GAP_DEGENERATE);
            const int ls = l - 1;
            const int hs = lane >> 3, ht = lane & 7;
            const auto full = [&](int t) { return t < dpos ? t : t + 1; };  // position in L
            if (ls > 0) {
                const T h2 = (hs < ls && ht < ls) ? S.post.Hs[full(hs) * SLM + full(ht)]
                                                  : num<T>::zero();
                if (!top_eig_h(h2, ls, hs, ht, lane, S.post.P, S.post.vs))
                    flags |= DIAF_FLAG_GAP_DEGENERATE;
            }
            T z = num<T>::zero();
            for (int t = 0; t < ls; ++t)
                z += num<T>::conj(S.post.vs[t]) * S.post.Hs[full(t) * SLM + dpos];
            const double az = num<T>::abs(z);
            const T e = az > 0.0 ? num<T>::div(z, az) : num<T>::one();
            if (lane < l)
                S.post.v[lane] = lane == dpos ? num<T>::mk(A.stab_r)
                                              : e * S.post.vs[lane < dpos ? lane : lane - 1];
            __syncthreads();
            if (lane < k) {
                T acc = num<T>::zero();
                for (int t = 0; t < l; ++t) acc += S.post.Y[lane * SLM + t] * S.post.v[t];
                S.post.w[lane] = acc;
            }
            __syncthreads();
        }
    }
    T res = num<T>::zero();
    if (lane < m)
        for (int pp = S.rptr[lane]; pp < S.rptr[lane + 1]; ++pp) {
            int e = S.csr[pp];
            res += S.eval[e] * S.post.w[S.ecol[e]];
        }
    for (int t = 0; t < l; ++t)
        if (S.L[t] == lane) res -= S.post.v[t];
    const double r2 = wave_sum(lane < m ? num<T>::abs2(res) : 0.0);
    if constexpr (MODE == 1) {
        // B without the rows of L (Bh) rank deficient: fewer rows than
        // columns, or its smallest singular value (the residual) negligible
        // against ||Bh||_F.  Its null space may then have dimension >= 2, where
        // the choice of w needs the eigenvectors of the generic kernel's
        // Jacobi solve: hand the column over.
        double f2 = 0.0;
        for (int t = lane; t < Tn; t += 64) {
            const int lr = S.eloc[t];
            bool inL = false;
            for (int q = 0; q < l; ++q) inL |= S.L[q] == lr;
            if (!inL) f2 += num<T>::abs2(S.eval[t]);
        }
        const double fro2 = wave_sum(f2);
        if (m - l < k || r2 <= 1e-14 * fro2) {
            __syncthreads();
            defer_push(db, j, lane, deferred, ndeferred);
            return;
        }
    }
    // ---- 10. outputs (V sorted by row) ----
    if (lane < k) A.Wval[jb + lane] = S.post.w[lane];
    int myL = lane < l ? S.L[lane] : 0x7fffffff;
    int rank = 0;
    for (int t = 0; t < l; ++t) rank += S.L[t] < myL;
    if (lane < l) {
        A.Vrows[(size_t)j * lmax + rank] = S.R[myL];
        A.Vvals[(size_t)j * lmax + rank] = S.post.v[lane];
    } else if (lane < lmax) {
        A.Vrows[(size_t)j * lmax + lane] = -1;
        A.Vvals[(size_t)j * lmax + lane] = num<T>::zero();
    }
    if (lane == 0) {
        A.rcol[j] = sqrt(r2);
        A.bnorm[j] = sqrt(bn2);
        A.flags[j] = flags;
        A.lcount[j] = l;
    }
    __syncthreads();
}

template <class T, int MODE>
__global__ void __launch_bounds__(64) factor_small_kernel(FactorArgs<T> A, int* deferred,
                                                          int* ndeferred)
{
    __shared__ SmallLds<T, MODE> S;
    // Workgroups are dealt to the 8 XCDs round robin by index; each XCD takes
    // a contiguous eighth of the column list, so neighbouring columns, which
    // gather overlapping columns of A, share an L2.  (Any dispatch order is
    // correct; this one only helps locality.)
    constexpr int NX = 8;
    const int nper = gridDim.x / NX;
    int q0 = blockIdx.x, qs = gridDim.x, qe = A.ncols;  // fewer than 8 workgroups: plain stride
    if (nper > 0) {
        if ((int)blockIdx.x >= nper * NX) return;
        const int x = blockIdx.x % NX, w = blockIdx.x / NX;
        const int chunk = (A.ncols + NX - 1) / NX;
        q0 = x * chunk + w;
        qs = nper;
        qe = min(A.ncols, (x + 1) * chunk);
    }
    // one call site, so the column body is inlined
    DeferBuf db;
    for (int q = q0; q < qe; q += qs) small_column(A, A.cols[q], S, deferred, ndeferred, db);
    defer_flush(db, threadIdx.x, deferred, ndeferred);
}

template <class T>
Err launch_factor_small(const FactorArgs<T>& A, int* deferred, int* ndeferred, FactorTune tune,
                        hipStream_t st)
{
    if (A.ncols == 0) return {};
    const int want = tune.small_grid > 0 ? tune.small_grid : 256 * 16;
    const int grid = A.ncols < want ? A.ncols : want;
    if (A.mode == 0)
        hipLaunchKernelGGL((factor_small_kernel<T, 0>), dim3(grid), dim3(64), 0, st, A, deferred,
                           ndeferred);
    else
        hipLaunchKernelGGL((factor_small_kernel<T, 1>), dim3(grid), dim3(64), 0, st, A, deferred,
                           ndeferred);
    DIAF_HIP_TRY(hipGetLastError());
    return {};
}

template <class T>
double small_occupancy(int mode)
{
    int nb = 0;
    const void* k = mode == 0 ? (const void*)factor_small_kernel<T, 0>
                              : (const void*)factor_small_kernel<T, 1>;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, 64, 0) != hipSuccess) return 0.0;
    return nb / 4.0;  // one wave per workgroup, four SIMDs per compute unit
}

template double small_occupancy<double>(int);
template double small_occupancy<zc>(int);

template Err launch_factor_small<double>(const FactorArgs<double>&, int*, int*, FactorTune,
                                         hipStream_t);
template Err launch_factor_small<zc>(const FactorArgs<zc>&, int*, int*, FactorTune, hipStream_t);

}  // namespace diaf
