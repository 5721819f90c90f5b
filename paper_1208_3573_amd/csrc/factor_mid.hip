// Mid-size column kernel for the first basic algorithm (unit-norm columns
// of V, paper Section 2.1): one wave per column for |J_j| <= MK (32 or 64)
// and at most MT (256, 512, 768 or 1024) gathered entries, so for shadows far
// beyond the one-wave kernel's 64 rows.  Columns it cannot take (more than
// 256 rows of B_j holding two or more entries, |L_j| > 8) are appended to a
// deferred list for the generic kernel.
//
// Per column j, with B = A(R_j, J_j) and G = B^* B:
//   * the gathered rows are deduplicated in an LDS hash table; the local id
//     of a row is its rank among the occupied slots.  No sort: every sum runs
//     over entries in their gathered order (column by column, rows ascending
//     within a column), so no result depends on the order of the local ids,
//     and ties in the V pattern are broken by global row;
//   * row access (CSR) from per-row counts, a wave scan and a per-row sort
//     of the entry ids (ascending entry = ascending column of B);
//   * G: the diagonal from each column's own entries; an off-diagonal entry
//     G(a, b) only for columns that share a row holding two or more entries
//     (per-column bit masks over these "shared rows", which are numbered
//     by ascending global row), summed over the common bits of the two
//     masks, i.e. over the shared rows in ascending global order;
//   * G = L L^* by a right-looking Cholesky in LDS, one lane per row;
//   * the seed w0 = G^{-1} b_j^* (V_0 = diagonals, Example 2.1), the scores
//     |(B w0)_i| of the admissible rows and the top-(l-1) selection with the
//     1e-10 tie band (Section 3.1), ties filled by ascending global row;
//   * Y = G^{-1} B_L^*, H = B_L Y (l x l) = M^* M for the paper's M_j
//     (eq. 2.3), v the top eigenvector of H by repeated squaring of the
//     trace-normalised power, w = Y v (eq. 2.4);
//   * phase (diagonal of V real positive), residual ||B w - v|| in FP64.
#include "dcommon.h"
#include "factor_kernels.h"

namespace diaf {
namespace mid {

constexpr int ML = 8;     // max |L_j| (and right-hand sides of a solve)
constexpr int MSW = 4;    // 64-bit words of a column's shared-row mask (256 shared rows)

// v of lane src (the same src on every lane) on every lane, by readlane
template <class T>
__device__ inline T bcast(T v, int src)
{
    if constexpr (num<T>::is_complex) return T{readlane_f64(v.x, src), readlane_f64(v.y, src)};
    else return readlane_f64(v, src);
}

// Whole-wave scan and reductions (every lane active): DPP and readlane,
// no LDS round trips.
__device__ inline int wave_incl_scan(int x, int) { return dpp_wave_incl_scan(x); }
__device__ inline double wave_sum(double x) { return dpp_wave_sum(x); }
__device__ inline double wave_max(double x) { return dpp_wave_max(x); }
__device__ inline int wave_min_int(int x) { return dpp_wave_min(x); }

// Packed lower triangle, row-major: G(i, q), q <= i.
__device__ inline int ltri(int i, int q) { return i * (i + 1) / 2 + q; }

constexpr int ilog2(int x) { return x <= 1 ? 0 : 1 + ilog2(x / 2); }
constexpr int pow2ceil(int x) { return x <= 1 ? 1 : 2 * pow2ceil((x + 1) / 2); }

template <class T, int MK, int MT>
struct MidLds {
    static constexpr int HS = pow2ceil(2 * MT);  // hash slots (load factor <= 1/2)
    static constexpr int HB = ilog2(HS);
    int a0[64];              // start of each column of B in A (lanes >= |J_j|: 0)
    int alen[64];            // and its length
    int hd[4];               // the column's j and the bounds of J_j in Jri
    int off[MK + 1];
    int R[MT];               // local row -> global row
    T eval[MT];              // gathered values, column by column
    uint8_t ecol[MT];        // column of B of each entry
    uint16_t eloc[MT];       // local row of each entry (first the hash slot)
    uint16_t rptr[MT + 1];   // CSR row starts
    uint16_t csr[MT];        // entry ids, row by row, ascending within a row
    uint16_t sidx[MT];       // shared-row index of a local row, 0xffff if single
    uint16_t she[MT];        // each column's entries in shared rows, in A's row order
    uint16_t soff[MK + 1];   // start of each column's list in she
    // storage reused by phase: the hash table (steps 2-4), the Gram matrix
    // and its Cholesky factor (steps 5-8), then the last step's vectors
    union {
        struct {
            int key[HS];  // hash keys (global rows), -1 empty; then each
                          // occupied slot's local row; then row counters
        } h;
        T G[MK * (MK + 1) / 2];  // packed lower triangle
        struct {
            T P[ML * ML];        // power of H being squared
            T v[ML];
            T w[MK];
        } f;
    };
    union {
        uint64_t cmask[MK][MSW];  // each column's shared rows (step 5)
        T X[MK][ML];              // right-hand sides and solutions (steps 7-8)
    };
    int L[ML];
};

// Top eigenvector of the Hermitian positive semidefinite l x l matrix (l <=
// 8) held one entry per lane (hs, ht) = (lane / 8, lane % 8), zero outside
// l x l: P = H / tr(H), then P <- P^2 / tr(P^2) (tr(P^2) = ||P||_F^2) until
// 1 - tr(P^2) < 1e-12, one squaring more, at most 25; the eigenvector is the
// column of the last power with the largest diagonal entry (lowest index on
// ties), normalised, into out[0..l).  Returns false when the trace is not
// positive or 25 squarings did not reach rank one (a relative gap below
// about 1e-6).
template <class T>
__device__ bool top_eig8(T h, int l, int hs, int ht, int lane, T* P, T* out)
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
        for (int q = 0; q < ML; ++q) acc += P[hs * ML + q] * P[q * ML + ht];
        __syncthreads();
        h = num<T>::div(acc, f);
    }
    if (!conv) ok = false;
    const double dg = (hs == ht && hs < l) ? num<T>::re(h) : -1.0;
    const double dmx = wave_max(dg);
    const uint64_t cm = __ballot(hs == ht && hs < l && dg == dmx);
    const int cstar = (__ffsll((unsigned long long)cm) - 1) >> 3;
    if (ht == cstar && hs < ML) out[hs] = h;
    __syncthreads();
    double nv = 0.0;
    for (int t = 0; t < l; ++t) nv += num<T>::abs2(out[t]);
    nv = sqrt(nv);
    __syncthreads();
    if (lane < l) out[lane] = num<T>::div(out[lane], nv);
    __syncthreads();
    return ok;
}

// Solve G X = X in place for nr right-hand sides (columns 0..nr-1 of S.X)
// with the Cholesky factor in S.G: forward L z = x, then backward L^* x = z.
// Lane i < k keeps row i of every right-hand side in registers; the pivot
// value of each step is broadcast by a shuffle.
template <class T, int MK, int MT>
__device__ void chol_solve(MidLds<T, MK, MT>& S, int k, int nr, int lane)
{
    T x[ML];
#pragma unroll
    for (int t = 0; t < ML; ++t)
        x[t] = (lane < k && t < nr) ? S.X[lane][t] : num<T>::zero();
    for (int p = 0; p < k; ++p) {
        const double d = num<T>::re(S.G[ltri(p, p)]);
        const double inv = d > 0.0 ? 1.0 / d : 0.0;
        const T lip = (lane > p && lane < k) ? S.G[ltri(lane, p)] : num<T>::zero();
#pragma unroll
        for (int t = 0; t < ML; ++t) {
            if (t >= nr) break;
            const T zp = num<T>::mk(inv) * bcast(x[t], p);
            if (lane == p) x[t] = zp;
            else if (lane > p) x[t] -= lip * zp;
        }
    }
    for (int p = k - 1; p >= 0; --p) {
        const double d = num<T>::re(S.G[ltri(p, p)]);
        const double inv = d > 0.0 ? 1.0 / d : 0.0;
        // conj(L(p, i)) for the lanes i < p: row p of L, contiguous
        const T lpi = lane < p ? num<T>::conj(S.G[ltri(p, lane)]) : num<T>::zero();
#pragma unroll
        for (int t = 0; t < ML; ++t) {
            if (t >= nr) break;
            const T xp = num<T>::mk(inv) * bcast(x[t], p);
            if (lane == p) x[t] = xp;
            else if (lane < p) x[t] -= lpi * xp;
        }
    }
#pragma unroll
    for (int t = 0; t < ML; ++t)
        if (lane < k && t < nr) S.X[lane][t] = x[t];
    __syncthreads();
}

// A column's head: j, the bounds of J_j in (Jcp, Jri) and, on lane a <
// min(|J_j|, MK), the bounds of column J_j[a] of A.  A wave loads the next
// column's head in three dependent steps spread over the current column
// (stage 1: J_j's bounds; 2: J_j; 3: A's column bounds) and publishes it to
// LDS (stage 4) before the current column's output stores, so the latency of
// that chain overlaps the current column's work.  The column numbers
// themselves come 64 at a time, one per lane, so between two columns no load
// is issued but at every 64th (a wait there would also wait for the stores
// just issued).
// Indices pass through a register the compiler cannot prove uniform, so
// these are vector loads: a pending scalar load would hold up every LDS
// wait.
struct MidHead {
    int j = -1, jb = 0, je = 0, c = 0, a0 = 0, a1 = 0, stage = 3;
};

__device__ inline void mid_head_start(MidHead& h, int j)
{
    h = MidHead{};
    h.j = j;
    h.stage = j >= 0 ? 0 : 3;
}

template <int MK, class T>
__device__ inline void mid_head_advance(const FactorArgs<T>& A, MidHead& h, int upto, int lane)
{
    if (h.stage >= upto) return;
    if (h.stage < 1) {
        int z = 0;
        __asm__ volatile("" : "+v"(z));
        h.jb = A.Jcp[h.j + z];
        h.je = A.Jcp[h.j + 1 + z];
    }
    if (h.stage < 2 && upto >= 2) {
        if (lane < h.je - h.jb && lane < MK) h.c = A.Jri[h.jb + lane];
    }
    if (h.stage < 3 && upto >= 3) {
        if (lane < h.je - h.jb && lane < MK) { h.a0 = A.Acp[h.c]; h.a1 = A.Acp[h.c + 1]; }
    }
    h.stage = upto;
}

template <int MK, class T, class S_t>
__device__ inline void mid_head_publish(const FactorArgs<T>& A, S_t& S, MidHead& h, int lane)
{
    if (h.stage == 4) return;
    mid_head_advance<MK>(A, h, 3, lane);
    // every load of the head completes here, on every path and lane
    __asm__ volatile("" ::"v"(h.j), "v"(h.jb), "v"(h.je), "v"(h.c), "v"(h.a0), "v"(h.a1));
    S.a0[lane] = h.a0;
    S.alen[lane] = h.a1 - h.a0;
    if (lane == 0) { S.hd[0] = h.j; S.hd[1] = h.jb; S.hd[2] = h.je; }
    h.stage = 4;
    __syncthreads();
}

template <class T, int MK, int MT>
__device__ void mid_column(const FactorArgs<T>& A, const int j, const int jb, const int k,
                           MidHead& nx, MidLds<T, MK, MT>& S, int* deferred, int* ndeferred)
{
    using S_t = MidLds<T, MK, MT>;
    constexpr int HS = S_t::HS;
    int lane = threadIdx.x;
    __asm__ volatile("" : "+v"(lane));
    const int lmax = A.lmax;
    const auto defer = [&]() {
        __syncthreads();
        if (lane == 0) deferred[atomicAdd(ndeferred, 1)] = j;
    };
    // ---- 1. J_j and gather offsets (k <= 64 = one lane per column) ----
    if (k > MK) { defer(); return; }
    const int len = lane < k ? S.alen[lane] : 0;
    const int inc = wave_incl_scan(len, lane);
    if (lane < k) S.off[lane + 1] = inc;
    if (lane == 0) S.off[0] = 0;
    const int Tn = __builtin_amdgcn_readlane(inc, 63);
    if (Tn > MT) { defer(); return; }
    for (int s = lane; s < HS; s += 64) S.h.key[s] = -1;
    __syncthreads();
    // ---- 2. gather; rows into the hash table ----
    // every load of this lane's entries (t = lane + 64 i) is issued before
    // the first is used, so the gather costs one memory latency, not MT / 64
    constexpr int EPL = MT / 64;
    int grow[EPL];
    T gval[EPL];
#pragma unroll
    for (int i = 0; i < EPL; ++i) {
        const int t = lane + 64 * i;
        grow[i] = 0;
        gval[i] = num<T>::zero();
        if (t < Tn) {
            int lo = 0, hi = k - 1;  // largest a with off[a] <= t
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (S.off[mid] <= t) lo = mid; else hi = mid - 1;
            }
            const int p = S.a0[lo] + (t - S.off[lo]);
            grow[i] = A.Ari[p];
            gval[i] = A.Aval[p];
            S.ecol[t] = (uint8_t)lo;
        }
    }
#pragma unroll
    for (int i = 0; i < EPL; ++i) {
        const int t = lane + 64 * i;
        if (t < Tn) {
            const int row = grow[i];
            S.eval[t] = gval[i];
            unsigned h = ((unsigned)row * 2654435761u) >> (32 - S_t::HB);  // < HS
            for (;;) {  // at most HS probes: the table is at most half full
                const int prev = atomicCAS(&S.h.key[h], -1, row);
                if (prev == -1 || prev == row) break;
                h = (h + 1) & (unsigned)(HS - 1);
            }
            S.eloc[t] = (uint16_t)h;
        }
    }
    __syncthreads();
    mid_head_advance<MK>(A, nx, 1, lane);
    // ---- 3. local rows: rank of each occupied slot ----
    int m = 0;
    for (int s0 = 0; s0 < HS; s0 += 64) {
        const int s = s0 + lane;
        const int key = S.h.key[s];
        const bool occ = key != -1;
        const uint64_t msk = __ballot(occ);
        const int pos = m + __popcll(msk & ((1ull << lane) - 1ull));
        if (occ) { S.R[pos] = key; S.h.key[s] = pos; }
        m += __popcll(msk);
    }
    __syncthreads();
    // m <= Tn <= MT: every row came from an entry
    for (int t = lane; t < Tn; t += 64) S.eloc[t] = (uint16_t)S.h.key[S.eloc[t]];
    for (int r = lane; r <= m; r += 64) S.rptr[r] = 0;
    int dj = -1;
    for (int r0 = 0; r0 < m; r0 += 64) {
        const uint64_t dm = __ballot(r0 + lane < m && S.R[r0 + lane] == j);
        if (dm && dj < 0) dj = r0 + __ffsll((unsigned long long)dm) - 1;
    }
    __syncthreads();
    // the hash table is dead from here: its keys' storage (HS >= 2 MT ints)
    // holds the row counters cnt[0..m) and cnt[MT..MT+m)
    int* cnt = S.h.key;
    for (int r = lane; r < m; r += 64) { cnt[r] = 0; cnt[MT + r] = 0; }
    __syncthreads();
    double bn2 = 0.0;
    for (int t = lane; t < Tn; t += 64) {
        atomicAdd(&cnt[S.eloc[t]], 1);
        bn2 += num<T>::abs2(S.eval[t]);
    }
    bn2 = wave_sum(bn2);
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
        __syncthreads();
        return;
    }
    // ---- 4. CSR by local row: exclusive scan of the counts, fill, sort ----
    {
        int base = 0;
        for (int r0 = 0; r0 < m; r0 += 64) {
            const int r = r0 + lane;
            const int c = r < m ? cnt[r] : 0;
            const int incl = wave_incl_scan(c, lane);
            if (r < m) S.rptr[r] = (uint16_t)(base + incl - c);
            base += __builtin_amdgcn_readlane(incl, 63);
        }
        if (lane == 0) S.rptr[m] = (uint16_t)Tn;
    }
    __syncthreads();
    for (int t = lane; t < Tn; t += 64) {
        const int r = S.eloc[t];
        const int pos = S.rptr[r] + atomicAdd(&cnt[MT + r], 1);
        S.csr[pos] = (uint16_t)t;
    }
    __syncthreads();
    int ms = 0;  // rows holding two or more entries ("shared rows")
    for (int r0 = 0; r0 < m; r0 += 64) {
        const int r = r0 + lane;
        bool sh = false;
        if (r < m) {
            const int b = S.rptr[r], e = S.rptr[r + 1];
            for (int p = b + 1; p < e; ++p) {  // ascending entry id = ascending column
                const uint16_t key = S.csr[p];
                int q = p - 1;
                while (q >= b && S.csr[q] > key) { S.csr[q + 1] = S.csr[q]; --q; }
                S.csr[q + 1] = key;
            }
            sh = e - b >= 2;
        }
        const uint64_t msk = __ballot(sh);
        const int qi = ms + __popcll(msk & ((1ull << lane) - 1ull));
        if (sh && qi < 64 * MSW) {  // list of the shared rows and their global rows
            S.she[qi] = (uint16_t)r;
            S.h.key[qi] = S.R[r];
        }
        ms += __popcll(msk);
    }
    if (ms > 64 * MSW) { defer(); return; }
    __syncthreads();
    // number the shared rows by ascending global row (rank among them), so
    // that walking a mask's bits upwards follows the rows of A in order
    {
        int key[MSW], rk[MSW];
#pragma unroll
        for (int i = 0; i < MSW; ++i) {
            key[i] = lane + 64 * i < ms ? S.h.key[lane + 64 * i] : 0x7fffffff;
            rk[i] = 0;
        }
        for (int u = 0; u < ms; ++u) {
            const int ku = S.h.key[u];
#pragma unroll
            for (int i = 0; i < MSW; ++i) rk[i] += ku < key[i];
        }
        for (int r = lane; r < m; r += 64) S.sidx[r] = (uint16_t)0xffff;
        __syncthreads();
#pragma unroll
        for (int i = 0; i < MSW; ++i)
            if (lane + 64 * i < ms) S.sidx[S.she[lane + 64 * i]] = (uint16_t)rk[i];
    }
    __syncthreads();
    // ---- 5. Gram matrix ----
    // lane a < k walks column a's entries (ascending global row): its mask
    // over the shared rows and its list of entries in shared rows (in the
    // order of the mask's bits)
    int ncs = 0;
    if (lane < k) {
        uint64_t mk_[MSW] = {};
        for (int t = S.off[lane]; t < S.off[lane + 1]; ++t) {
            const int q = S.sidx[S.eloc[t]];
            if (q != 0xffff) {
                mk_[q >> 6] |= 1ull << (q & 63);
                ++ncs;
            }
        }
#pragma unroll
        for (int wd = 0; wd < MSW; ++wd) S.cmask[lane][wd] = mk_[wd];
    }
    {
        const int incl = wave_incl_scan(ncs, lane);
        if (lane < k) S.soff[lane] = (uint16_t)(incl - ncs);
        if (lane == k - 1) S.soff[k] = (uint16_t)incl;
        __syncthreads();
        if (lane < k) {
            int pos = incl - ncs;
            for (int t = S.off[lane]; t < S.off[lane + 1]; ++t)
                if (S.sidx[S.eloc[t]] != 0xffff) S.she[pos++] = (uint16_t)t;
        }
    }
    T dg = num<T>::zero();
    if (lane < k)
        for (int t = S.off[lane]; t < S.off[lane + 1]; ++t)
            dg += num<T>::cmul(S.eval[t], S.eval[t]);
    const double maxd = wave_max(lane < k ? num<T>::re(dg) : 0.0);
    __syncthreads();  // the hash table's storage becomes G
    if (lane < k) S.G[ltri(lane, lane)] = dg;
    {
        const int npair = k * (k - 1) / 2;
        for (int pi = lane; pi < npair; pi += 64) {
            // strictly lower pair: pi = a (a - 1) / 2 + b, b < a
            int a = (int)((sqrtf(8.0f * (float)pi + 1.0f) + 1.0f) * 0.5f);
            while (a * (a - 1) / 2 > pi) --a;
            while ((a + 1) * a / 2 <= pi) ++a;
            const int b = pi - a * (a - 1) / 2;
            // the shared rows of both columns are the common bits of their
            // masks; walking them upwards sums over the rows in ascending
            // global order, so the sum does not depend on the local row ids.
            // A column's entry at shared row q is its list entry number
            // (mask bits below q).
            T acc = num<T>::zero();
            int ba = S.soff[a], bb = S.soff[b];
#pragma unroll
            for (int wd = 0; wd < MSW; ++wd) {
                const uint64_t ma = S.cmask[a][wd], mb = S.cmask[b][wd];
                uint64_t cm = ma & mb;
                while (cm) {
                    const uint64_t below = (cm & (~cm + 1ull)) - 1ull;
                    cm &= cm - 1ull;
                    const int ta = S.she[ba + __popcll(ma & below)];
                    const int tb = S.she[bb + __popcll(mb & below)];
                    acc += num<T>::cmul(S.eval[ta], S.eval[tb]);  // conj(B(r, a)) B(r, b)
                }
                ba += __popcll(ma);
                bb += __popcll(mb);
            }
            S.G[ltri(a, b)] = acc;
        }
    }
    __syncthreads();
    mid_head_advance<MK>(A, nx, 2, lane);
    // ---- 6. Cholesky G = L L^*, left-looking, one lane per row ----
    // step p: every row i >= p takes G(i, p) - sum_{q<p} L(i, q) conj(L(p, q))
    // (independent loads of its own row and of row p); row p's value is the
    // pivot, the rows below divide by its square root
    uint32_t flags = 0;
    if (k > m) flags |= DIAF_FLAG_RANK_DEFICIENT;
    for (int p = 0; p < k; ++p) {
        T sp = num<T>::zero();
        if (lane >= p && lane < k) {
            sp = S.G[ltri(lane, p)];
            // four terms at a time: their loads in flight together, the
            // subtractions in ascending q as one at a time would do them
            const T* gi = S.G + ltri(lane, 0);
            const T* gp = S.G + ltri(p, 0);
            int q = 0;
            for (; q + 4 <= p; q += 4) {
                const T a0 = gi[q], a1 = gi[q + 1], a2 = gi[q + 2], a3 = gi[q + 3];
                const T b0 = gp[q], b1 = gp[q + 1], b2 = gp[q + 2], b3 = gp[q + 3];
                sp -= a0 * num<T>::conj(b0);
                sp -= a1 * num<T>::conj(b1);
                sp -= a2 * num<T>::conj(b2);
                sp -= a3 * num<T>::conj(b3);
            }
            for (; q < p; ++q) sp -= gi[q] * num<T>::conj(gp[q]);
        }
        const double d = num<T>::re(bcast(sp, p));
        if (!(d > 1e-14 * maxd)) flags |= DIAF_FLAG_RANK_DEFICIENT;
        const double piv = (d > 1e-30 * maxd && isfinite(d)) ? sqrt(d) : 0.0;
        const double inv = piv > 0.0 ? 1.0 / piv : 0.0;
        if (lane == p) S.G[ltri(p, p)] = num<T>::mk(piv);
        else if (lane > p && lane < k) S.G[ltri(lane, p)] = num<T>::mk(inv) * sp;
        __syncthreads();
    }
    mid_head_advance<MK>(A, nx, 3, lane);
    // ---- 7. V pattern ----
    const bool topk =
        A.vrule == V_TOPK_LOWER || A.vrule == V_TOPK_UPPER || A.vrule == V_TOPK_BLOCK;
    int l = 0;
    if (topk) {
        if (lane < k) S.X[lane][0] = num<T>::zero();
        __syncthreads();
        for (int pp = S.rptr[dj] + lane; pp < S.rptr[dj + 1]; pp += 64) {
            const int e = S.csr[pp];
            S.X[S.ecol[e]][0] = num<T>::conj(S.eval[e]);
        }
        __syncthreads();
        chol_solve(S, k, 1, lane);  // w0 = G^{-1} b_j^*
        const int blo = A.vrule == V_TOPK_BLOCK ? A.vblk[2 * j] : 0;
        const int bhi = A.vrule == V_TOPK_BLOCK ? A.vblk[2 * j + 1] : 0;
        // scores of this lane's rows r = lane + 64 i in registers (-1: not
        // admissible)
        constexpr int RPL = MT / 64;
        double sc[RPL];
        int ncl = 0;
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
            const int r = lane + 64 * i;
            double s = -1.0;
            if (r < m) {
                const int gi = S.R[r];
                const bool adm = A.vrule == V_TOPK_BLOCK ? (gi != j && gi >= blo && gi < bhi)
                                 : A.vrule == V_TOPK_LOWER ? gi > j : gi < j;
                if (adm) {
                    T y = num<T>::zero();
                    for (int pp = S.rptr[r]; pp < S.rptr[r + 1]; ++pp) {
                        const int e = S.csr[pp];
                        y += S.eval[e] * S.X[S.ecol[e]][0];
                    }
                    s = num<T>::abs(y);
                    ++ncl;
                }
            }
            sc[i] = s;
        }
        const int nc = (int)wave_sum((double)ncl);
        int lj = A.vcount < 1 ? 1 : A.vcount;
        if (lj > 1 + nc) lj = 1 + nc;
        if (lj > lmax) lj = lmax;
        if (lj > ML) lj = ML;
        const int q = lj - 1;
        // bit i of these masks: row lane + 64 i
        uint32_t chosen = 0;
        if (q > 0 && nc <= q) {
#pragma unroll
            for (int i = 0; i < RPL; ++i)
                if (sc[i] >= 0.0) chosen |= 1u << i;
        } else if (q > 0) {
            // the q-th largest score, counting equal scores separately
            uint32_t taken = 0;
            double ss = 0.0;
            for (int rd = 0; rd < q; ++rd) {
                double best = -2.0;
                int bi = -1;
#pragma unroll
                for (int i = 0; i < RPL; ++i)
                    if (sc[i] >= 0.0 && !((taken >> i) & 1u) && sc[i] > best) {
                        best = sc[i];
                        bi = i;
                    }
                const double mx = wave_max(best);
                const uint64_t bm = __ballot(best == mx && bi >= 0);
                if (lane == __ffsll((unsigned long long)bm) - 1) taken |= 1u << bi;
                ss = mx;
            }
            const double hi = ss * (1.0 + 1e-10), lo = ss * (1.0 - 1e-10);
            uint32_t tie = 0;
            int nin = 0;
            bool edge = false;
#pragma unroll
            for (int i = 0; i < RPL; ++i) {
                const double sv = sc[i];
                if (sv < 0.0) continue;
                if (sv > hi) { chosen |= 1u << i; ++nin; }
                else if (sv >= lo) tie |= 1u << i;
                if (ss > 0.0 && (fabs(sv - hi) <= 1e-12 * ss || fabs(sv - lo) <= 1e-12 * ss))
                    edge = true;
            }
            if (__ballot(edge)) flags |= DIAF_FLAG_TIE_EDGE;
            int need = q - (int)wave_sum((double)nin);
            // fill the tie class by ascending global row
            for (; need > 0; --need) {
                int gbest = 0x7fffffff, ib = -1;
                for (int i = 0; lane + 64 * i < m; ++i)
                    if (((tie >> i) & 1u) && S.R[lane + 64 * i] < gbest) {
                        gbest = S.R[lane + 64 * i];
                        ib = i;
                    }
                const int gm = wave_min_int(gbest);
                if (gm == 0x7fffffff) break;
                if (ib >= 0 && gbest == gm) { chosen |= 1u << ib; tie &= ~(1u << ib); }
            }
        }
        // compact: L[0] = j's row, then the chosen rows
        l = 1;
        for (int i = 0; i < MT / 64; ++i) {
            const bool c = (chosen >> i) & 1u;
            const uint64_t cm = __ballot(c);
            if (c) S.L[l + __popcll(cm & ((1ull << lane) - 1ull))] = lane + 64 * i;
            l += __popcll(cm);
        }
        if (lane == 0) S.L[0] = dj;
    } else if (A.vrule == V_DIAG) {
        if (lane == 0) S.L[0] = dj;
        l = 1;
    } else {
        // Gauss-Seidel structure or an explicit pattern: the listed rows of
        // column j that lie in the shadow, found by a scan of R
        int b = 0, e = 0;
        const int32_t* rows = nullptr;
        if (A.vrule == V_EXPLICIT) { b = A.Vcp_in[j]; e = A.Vcp_in[j + 1]; rows = A.Vri_in; }
        else { b = A.Acp[j]; e = A.Acp[j + 1]; rows = A.Ari; }
        for (int p = b; p < e; ++p) {
            const int gi = rows[p];
            const bool keep = A.vrule == V_EXPLICIT || gi == j ||
                              (A.vrule == V_GS_UPPER ? gi < j : gi > j);
            if (!keep) continue;
            int lr = -1;
            for (int r0 = 0; r0 < m && lr < 0; r0 += 64) {
                const uint64_t hm = __ballot(r0 + lane < m && S.R[r0 + lane] == gi);
                if (hm) lr = r0 + __ffsll((unsigned long long)hm) - 1;
            }
            if (lr < 0) continue;
            if (l < ML && lane == 0) S.L[l] = lr;
            ++l;
        }
        if (l > ML || l > lmax) { defer(); return; }
    }
    __syncthreads();
    // ---- 8. Y = G^{-1} B_L^*, H = B_L Y, v = top eigenvector of H, w = Y v ----
    if (lane < k) {
#pragma unroll
        for (int t = 0; t < ML; ++t) S.X[lane][t] = num<T>::zero();
    }
    __syncthreads();
    for (int t = 0; t < l; ++t) {
        const int r = S.L[t];
        for (int pp = S.rptr[r] + lane; pp < S.rptr[r + 1]; pp += 64) {
            const int e = S.csr[pp];
            S.X[S.ecol[e]][t] = num<T>::conj(S.eval[e]);
        }
    }
    __syncthreads();
    chol_solve(S, k, l, lane);
    {
        const int hs = lane >> 3, ht = lane & 7;
        T h = num<T>::zero();
        if (hs < l && ht < l) {
            const int r = S.L[hs];
            for (int pp = S.rptr[r]; pp < S.rptr[r + 1]; ++pp) {
                const int e = S.csr[pp];
                h += S.eval[e] * S.X[S.ecol[e]][ht];
            }
        }
        __syncthreads();  // G is dead: its storage holds P, v and w
        if (!top_eig8(h, l, hs, ht, lane, S.f.P, S.f.v)) flags |= DIAF_FLAG_GAP_DEGENERATE;
    }
    if (lane < k) {
        T acc = num<T>::zero();
        for (int t = 0; t < l; ++t) acc += S.X[lane][t] * S.f.v[t];
        S.f.w[lane] = acc;
    }
    __syncthreads();
    // ---- 9. phase, residual, outputs ----
    T vt = lane < l ? S.f.v[lane] : num<T>::zero();
    const double vn = sqrt(wave_sum(lane < l ? num<T>::abs2(vt) : 0.0));
    const uint64_t dposm = __ballot(lane < l && S.L[lane] == dj);
    const int dpos = dposm ? __ffsll((unsigned long long)dposm) - 1 : -1;
    int piv;
    if (dpos >= 0 && num<T>::abs(bcast(vt, dpos)) >= 1e-8 * vn) {
        piv = dpos;
    } else {
        const double av = lane < l ? num<T>::abs(vt) : -1.0;
        const double mx = wave_max(av);
        const int gr = lane < l ? S.R[S.L[lane]] : 0x7fffffff;
        const int cand = wave_min_int((lane < l && av == mx) ? gr : 0x7fffffff);
        const uint64_t pm = __ballot(lane < l && av == mx && gr == cand);
        piv = __ffsll((unsigned long long)pm) - 1;
    }
    const T pvv = bcast(vt, piv);
    const T ph = num<T>::iszero(pvv) ? num<T>::one() : unit_conj_phase(pvv);
    vt = ph * vt;
    if (dpos < 0 || num<T>::abs(bcast(vt, dpos < 0 ? 0 : dpos)) < 1e-2 * vn)
        flags |= DIAF_FLAG_SMALL_DIAG;
    if (lane < l) S.f.v[lane] = vt;
    if (lane < k) S.f.w[lane] = ph * S.f.w[lane];
    __syncthreads();
    // residual: each row is taken by the lane of its first entry, so the
    // order of the sum follows the entries, not the local row ids
    double r2 = 0.0;
    for (int t0 = lane; t0 < Tn; t0 += 64) {
        const int r = S.eloc[t0];
        if (S.csr[S.rptr[r]] != t0) continue;
        T res = num<T>::zero();
        for (int pp = S.rptr[r]; pp < S.rptr[r + 1]; ++pp) {
            const int e = S.csr[pp];
            res += S.eval[e] * S.f.w[S.ecol[e]];
        }
        for (int t = 0; t < l; ++t)
            if (S.L[t] == r) res -= S.f.v[t];
        r2 += num<T>::abs2(res);
    }
    r2 = wave_sum(r2);
    mid_head_publish<MK>(A, S, nx, lane);  // S.a0, S.alen and S.hd are dead here
    if (lane < k) A.Wval[jb + lane] = S.f.w[lane];
    const int myg = lane < l ? S.R[S.L[lane]] : 0x7fffffff;
    int rank = 0;
    for (int t = 0; t < l; ++t) rank += S.R[S.L[t]] < myg;
    if (lane < l) {
        A.Vrows[(size_t)j * lmax + rank] = myg;
        A.Vvals[(size_t)j * lmax + rank] = S.f.v[lane];
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

template <class T, int MK, int MT>
__global__ void __launch_bounds__(64) factor_mid_kernel(FactorArgs<T> A, int* deferred,
                                                        int* ndeferred)
{
    __shared__ MidLds<T, MK, MT> S;
    // contiguous eighths of the column list per XCD (workgroups are dealt to
    // the 8 XCDs round robin), as in the one-wave kernel
    constexpr int NX = 8;
    const int nper = gridDim.x / NX;
    int q0 = blockIdx.x, qs = gridDim.x, qe = A.ncols;
    if (nper > 0) {
        if ((int)blockIdx.x >= nper * NX) return;
        const int x = blockIdx.x % NX, w = blockIdx.x / NX;
        const int chunk = (A.ncols + NX - 1) / NX;
        q0 = x * chunk + w;
        qs = nper;
        qe = min(A.ncols, (x + 1) * chunk);
    }
    const int lane = threadIdx.x;
    // colv on lane i: the column of iteration 64 b + i of this wave (-1 past
    // the end), for the current block b of 64 iterations
    const auto col_block = [&](int it0) {
        const int q = q0 + (it0 + lane) * qs;
        return q < qe ? A.cols[q] : -1;
    };
    int colv = col_block(0);
    MidHead nx;
    mid_head_start(nx, __builtin_amdgcn_readlane(colv, 0));
    mid_head_publish<MK>(A, S, nx, lane);
    for (int it = 0, q = q0; q < qe; ++it, q += qs) {
        // this column's head, from LDS; the next column's number, from colv
        const int j = __builtin_amdgcn_readfirstlane(S.hd[0]);
        const int jb = __builtin_amdgcn_readfirstlane(S.hd[1]);
        const int k = __builtin_amdgcn_readfirstlane(S.hd[2]) - jb;
        if (((it + 1) & 63) == 0) colv = col_block(it + 1);
        mid_head_start(nx, __builtin_amdgcn_readlane(colv, (it + 1) & 63));
        mid_column(A, j, jb, k, nx, S, deferred, ndeferred);
        mid_head_publish<MK>(A, S, nx, lane);
    }
}

}  // namespace mid

template <class T>
bool mid_supports(int kcap, int tcap)
{
    if constexpr (num<T>::is_complex) return kcap <= 32 && tcap <= 256;
    else return kcap <= 64 && tcap <= 1024;
}

template <class T>
int mid_classes(int* kcap, int* tcap)
{
    // capacities of the kernel instances, smallest LDS first (a column takes
    // the first that holds it)
    static const int cls[][2] = {{32, 256}, {32, 512}, {64, 512}, {32, 1024}, {64, 768},
                                 {64, 1024}};
    const int nc = num<T>::is_complex ? 1 : 6;
    for (int c = 0; c < nc; ++c) { kcap[c] = cls[c][0]; tcap[c] = cls[c][1]; }
    return nc;
}

template <class T, int MK, int MT>
static Err launch_mid_t(const FactorArgs<T>& A, int* deferred, int* ndeferred, int grid,
                        hipStream_t st)
{
    hipLaunchKernelGGL((mid::factor_mid_kernel<T, MK, MT>), dim3(grid), dim3(64), 0, st, A,
                       deferred, ndeferred);
    DIAF_HIP_TRY(hipGetLastError());
    return {};
}

template <class T>
Err launch_factor_mid(const FactorArgs<T>& A, int kcap, int tcap, int* deferred, int* ndeferred,
                      FactorTune tune, hipStream_t st)
{
    if (A.ncols == 0) return {};
    if (!mid_supports<T>(kcap, tcap)) return {DIAF_EINVAL, "mid kernel: size class too large"};
    const int want = tune.small_grid > 0 ? tune.small_grid : 256 * 16;
    const int grid = A.ncols < want ? A.ncols : want;
    if (kcap <= 32 && tcap <= 256) return launch_mid_t<T, 32, 256>(A, deferred, ndeferred, grid, st);
    if constexpr (!num<T>::is_complex) {
        if (kcap <= 32 && tcap <= 512) return launch_mid_t<T, 32, 512>(A, deferred, ndeferred, grid, st);
        if (tcap <= 512) return launch_mid_t<T, 64, 512>(A, deferred, ndeferred, grid, st);
        if (kcap <= 32) return launch_mid_t<T, 32, 1024>(A, deferred, ndeferred, grid, st);
        if (tcap <= 768) return launch_mid_t<T, 64, 768>(A, deferred, ndeferred, grid, st);
        return launch_mid_t<T, 64, 1024>(A, deferred, ndeferred, grid, st);
    }
    return {DIAF_EINVAL, "mid kernel: size class too large"};
}

template <class T>
double mid_occupancy(int kcap, int tcap)
{
    int nb = 0;
    const void* k = nullptr;
    if (kcap <= 32 && tcap <= 256) k = (const void*)mid::factor_mid_kernel<T, 32, 256>;
    if constexpr (!num<T>::is_complex) {
        if (!k && kcap <= 32 && tcap <= 512) k = (const void*)mid::factor_mid_kernel<T, 32, 512>;
        if (!k && tcap <= 512) k = (const void*)mid::factor_mid_kernel<T, 64, 512>;
        if (!k && kcap <= 32) k = (const void*)mid::factor_mid_kernel<T, 32, 1024>;
        if (!k && tcap <= 768) k = (const void*)mid::factor_mid_kernel<T, 64, 768>;
        if (!k) k = (const void*)mid::factor_mid_kernel<T, 64, 1024>;
    }
    if (!k || hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, 64, 0) != hipSuccess) return 0.0;
    return nb / 4.0;
}

template bool mid_supports<double>(int, int);
template bool mid_supports<zc>(int, int);
template int mid_classes<double>(int*, int*);
template int mid_classes<zc>(int*, int*);
template Err launch_factor_mid<double>(const FactorArgs<double>&, int, int, int*, int*, FactorTune,
                                       hipStream_t);
template Err launch_factor_mid<zc>(const FactorArgs<zc>&, int, int, int*, int*, FactorTune,
                                   hipStream_t);
template double mid_occupancy<double>(int, int);
template double mid_occupancy<zc>(int, int);

}  // namespace diaf
