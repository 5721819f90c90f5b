// W pattern by sparsified powers (paper Section 4, Algorithm 1), real or
// complex A, with V_0 the diagonal or the block diagonal matrices.
//
// The splitting A = V_0 (I - S), V_0 = P_{V_0} A, gives S = V_0^{-1}(A -
// P_{V_0} A).  With V_0 = diag(A), S(i, c) = a_ic / a_ii off the diagonal.
// With V_0 block diagonal (blocks of consecutive rows and columns, at most
// 64), V_0 is A's block diagonal part, each block is factored once (partial
// pivoting, by the block-V LU kernel), and column c of S is the block solve
// of A(:, c) outside c's block: every row of every block it reaches is an
// entry of S.  The columns of S are sparsified once (tolerance tau_i
// relative to the column's largest entry, then at most p_i entries, the
// largest); then, for every column j, t = e_j is multiplied by S k times,
// each product sparsified by (tau_l, p_l) with row j exempt, and the pattern
// of w_j is the union of e_j and every kept t (the truncated series I + S +
// ... + S^k taken entry by entry), less the rows of j's block other than j
// (the algorithm's final removal of V_0 minus the identity; nothing for the
// diagonal V_0).
//
// Reading of the dropping rules (the paper fixes neither the norm nor the
// tie order): magnitudes are compared as squares |v|^2 (v*v, or re*re +
// im*im), the tolerance test is |v|^2 >= (tau*tau) * max |v|^2 over the
// vector (row j included for t), a zero parameter disables its rule, and
// among entries of equal magnitude the count rule keeps the lower rows.
// Products are formed and summed per output row in ascending source row
// with explicit round-to-nearest operations (complex products as
// (ar br - ai bi, ar bi + ai br), the division by a diagonal entry as
// a conj(d) / |d|^2), so with the diagonal V_0 every value, and hence every
// dropping decision, is reproducible bit for bit.
//
// Kernels: a diagonal gather; one wave per column of S for the scaling (or
// the block solves) and the initial dropping (entries staged in LDS); one
// wave per column j for the level expansion.  The expansion walks the
// sources of t in ascending row, one after the other; the entries of one
// column of S go to the 64 lanes, whose rows are distinct, into an LDS hash
// accumulator (row -> slot, insertion by compare-and-swap), so per output
// row the partial sums arrive in source order.  The accumulated rows are
// then ranked into ascending order, dropped and compacted in place, and
// added to an LDS hash set that holds the pattern of s_j.  Two LDS sizes are
// built; columns that outgrow the smaller one are listed and rerun with the
// larger one.
#include "dcommon.h"
#include "factor_kernels.h"

namespace diaf {

namespace {

constexpr int SB_CAP = 1024;  // entries of one column of S staged in LDS

// Arithmetic with the rounding spelled out (no contraction).
__device__ inline double sqm(double v) { return __dmul_rn(v, v); }
__device__ inline double sqm(zc v) { return __dadd_rn(__dmul_rn(v.x, v.x), __dmul_rn(v.y, v.y)); }
__device__ inline double mul_rn(double a, double b) { return __dmul_rn(a, b); }
__device__ inline zc mul_rn(zc a, zc b)
{
    return {__dsub_rn(__dmul_rn(a.x, b.x), __dmul_rn(a.y, b.y)),
            __dadd_rn(__dmul_rn(a.x, b.y), __dmul_rn(a.y, b.x))};
}
__device__ inline double add_rn(double a, double b) { return __dadd_rn(a, b); }
__device__ inline zc add_rn(zc a, zc b) { return {__dadd_rn(a.x, b.x), __dadd_rn(a.y, b.y)}; }
__device__ inline double div_rn(double a, double d) { return __ddiv_rn(a, d); }
__device__ inline zc div_rn(zc a, zc d)
{
    const double den = __dadd_rn(__dmul_rn(d.x, d.x), __dmul_rn(d.y, d.y));
    return {__ddiv_rn(__dadd_rn(__dmul_rn(a.x, d.x), __dmul_rn(a.y, d.y)), den),
            __ddiv_rn(__dsub_rn(__dmul_rn(a.y, d.x), __dmul_rn(a.x, d.y)), den)};
}
__device__ inline double spshfl(double v, int src) { return __shfl(v, src); }
__device__ inline zc spshfl(zc v, int src) { return {__shfl(v.x, src), __shfl(v.y, src)}; }
__device__ inline double spdiv(double a, double b) { return a / b; }
__device__ inline zc spdiv(zc a, zc b)
{
    const double d = b.x * b.x + b.y * b.y;
    return {(a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d};
}

__device__ inline double wave_max(double v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}

__device__ inline int wave_sum(int v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__device__ inline uint64_t lanes_below(int lane) { return (1ull << lane) - 1ull; }

// Slot of key in an LDS open-addressing table of HC slots (empty = -1),
// inserting it when absent; -1 when the table is full.
template <int HC>
__device__ inline int hash_slot(int32_t* keys, int key, bool& inserted)
{
    unsigned h = ((unsigned)key * 2654435761u) & (HC - 1);
    for (int probe = 0; probe < HC; ++probe) {
        int old = atomicCAS(&keys[h], -1, key);
        if (old == -1) {
            inserted = true;
            return (int)h;
        }
        if (old == key) {
            inserted = false;
            return (int)h;
        }
        h = (h + 1) & (HC - 1);
    }
    inserted = false;
    return -1;
}

// Initial dropping of one column of S staged in LDS (rw: rows ascending, -1
// for a position that is no entry; vl: values), by (tau, p); the kept
// entries are written in order to dst_r / dst_v (when dst_r is given);
// returns their number (every lane).
template <class T>
__device__ int drop_staged(const int32_t* rw, const T* vl, int na, double tau, int p, int lane,
                           int32_t* dst_r, T* dst_v)
{
    double mx = 0.0;
    for (int q = lane; q < na; q += 64)
        if (rw[q] >= 0) mx = fmax(mx, sqm(vl[q]));
    mx = wave_max(mx);
    const double thr = tau > 0.0 ? __dmul_rn(__dmul_rn(tau, tau), mx) : 0.0;
    int ncand = 0;
    for (int q = lane; q < na; q += 64) ncand += rw[q] >= 0 && (tau <= 0.0 || sqm(vl[q]) >= thr);
    ncand = wave_sum(ncand);
    const bool by_count = p > 0 && ncand > p;
    int base = 0;
    for (int q0 = 0; q0 < na; q0 += 64) {
        const int q = q0 + lane;
        bool keep = false;
        int row = -1;
        T v = num<T>::zero();
        if (q < na) {
            row = rw[q];
            v = vl[q];
            const double m = sqm(v);
            keep = row >= 0 && (tau <= 0.0 || m >= thr);
            if (keep && by_count) {
                int rank = 0;
                for (int f = 0; f < na; ++f) {
                    const int rf = rw[f];
                    if (rf < 0) continue;
                    const double mf = sqm(vl[f]);
                    if (tau > 0.0 && mf < thr) continue;
                    rank += mf > m || (mf == m && rf < row);
                }
                keep = rank < p;
            }
        }
        const uint64_t bal = __ballot(keep);
        if (keep && dst_r) {
            const int pos = base + __popcll(bal & lanes_below(lane));
            dst_r[pos] = row;
            dst_v[pos] = v;
        }
        base += __popcll(bal);
    }
    return base;
}

}  // namespace

// d[c] = a_cc (columns of A have their diagonal; validated before).  Bit 0
// of *bad is set for a zero diagonal.
template <class T>
__global__ void sp_diag_kernel(int n, const int32_t* Acp, const int32_t* Ari, const T* Aval, T* d,
                               int32_t* bad)
{
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    T v = num<T>::zero();
    for (int q = Acp[c]; q < Acp[c + 1]; ++q)
        if (Ari[q] == c) {
            v = Aval[q];
            break;
        }
    d[c] = v;
    if (num<T>::iszero(v)) atomicOr(bad, 1);
}

// Column c of S for the diagonal V_0, sparsified by (tau, p), written at
// Acp[c] .. Acp[c] + scnt[c] of Sri/Sval with ascending rows.  Bit 1 of
// *bad is set for a column of A longer than SB_CAP.
template <class T>
__global__ __launch_bounds__(64) void sp_build_s_kernel(int n, const int32_t* Acp,
                                                        const int32_t* Ari, const T* Aval,
                                                        const T* d, double tau, int p,
                                                        int32_t* Sri, T* Sval, int32_t* scnt,
                                                        int32_t* bad)
{
    __shared__ int32_t rw[SB_CAP];
    __shared__ T vl[SB_CAP];
    const int c = blockIdx.x;
    const int lane = threadIdx.x;
    const int a0 = Acp[c], na = Acp[c + 1] - a0;
    if (na > SB_CAP) {
        if (lane == 0) {
            scnt[c] = 0;
            atomicOr(bad, 2);
        }
        return;
    }
    for (int q = lane; q < na; q += 64) {
        const int i = Ari[a0 + q];
        rw[q] = i == c ? -1 : i;  // the diagonal of A is not an entry of S
        vl[q] = i == c ? num<T>::zero() : div_rn(Aval[a0 + q], d[i]);
    }
    __syncthreads();
    const int cnt = drop_staged(rw, vl, na, tau, p, lane, Sri + a0, Sval + a0);
    if (lane == 0) scnt[c] = cnt;
}

// D = A's block diagonal part (V_0 = P_{V_0} A) in CSC: count pass (Dri
// null) or fill pass.  rb: per row, its block's rows [rb[2i], rb[2i+1]).
template <class T>
__global__ void sp_block_d_kernel(int n, const int32_t* Acp, const int32_t* Ari, const T* Aval,
                                  const int32_t* rb, int32_t* cnt, const int32_t* Dcp,
                                  int32_t* Dri, T* Dval)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const int lo = rb[2 * j], hi = rb[2 * j + 1];
    int c = 0;
    for (int p = Acp[j]; p < Acp[j + 1]; ++p) {
        const int i = Ari[p];
        if (i >= lo && i < hi) {
            if (Dri) {
                Dri[Dcp[j] + c] = i;
                Dval[Dcp[j] + c] = Aval[p];
            }
            ++c;
        }
    }
    if (!Dri) cnt[j] = c;
}

// Column c of S for the block diagonal V_0: the entries of A(:, c) outside
// c's block, grouped by the block of their row (rows ascending), each group
// solved with that block's LU factors (LU + boff[b], column-major, row
// permutation perm[bstart[b] ..]; lane i holds row i of the block), then
// sparsified by (tau, p).  Count pass (Sri null): scnt[c]; fill pass: the
// entries at Scp[c].  Bit 1 of *bad: more than SB_CAP staged entries.
template <class T>
__global__ __launch_bounds__(64) void sp_build_s_block_kernel(
    int n, const int32_t* Acp, const int32_t* Ari, const T* Aval, const int32_t* rb,
    const int32_t* bid, const int32_t* bstart, const int64_t* boff, const T* LU,
    const int32_t* perm, double tau, int p, int32_t* scnt, const int32_t* Scp, int32_t* Sri,
    T* Sval, int32_t* bad)
{
    __shared__ int32_t rw[SB_CAP];
    __shared__ T vl[SB_CAP];
    __shared__ int32_t er[SB_CAP];  // A's entries of column c outside c's block
    __shared__ T ev[SB_CAP];
    const int c = blockIdx.x;
    const int lane = threadIdx.x;
    const int a0 = Acp[c], na = Acp[c + 1] - a0;
    const int clo = rb[2 * c], chi = rb[2 * c + 1];
    if (na > SB_CAP) {
        if (lane == 0) {
            if (!Sri) scnt[c] = 0;
            atomicOr(bad, 2);
        }
        return;
    }
    // stage the entries outside c's block, ascending rows
    int ne = 0;
    for (int q0 = 0; q0 < na; q0 += 64) {
        const int q = q0 + lane;
        const int i = q < na ? Ari[a0 + q] : -1;
        const bool out = q < na && (i < clo || i >= chi);
        const uint64_t bal = __ballot(out);
        if (out) {
            const int pos = ne + __popcll(bal & lanes_below(lane));
            er[pos] = i;
            ev[pos] = Aval[a0 + q];
        }
        ne += __popcll(bal);
    }
    __syncthreads();
    // one block solve per run of entries in the same block
    int nst = 0;
    bool over = false;
    for (int t = 0; t < ne;) {
        const int b = bid[er[t]];
        const int b0 = bstart[b], bs = bstart[b + 1] - b0;
        int t2 = t;
        while (t2 < ne && er[t2] < b0 + bs) ++t2;
        if (nst + bs > SB_CAP) {
            over = true;
            break;
        }
        T r = num<T>::zero();
        for (int u = t; u < t2; ++u)
            if (er[u] - b0 == lane) r = ev[u];
        const T* F = LU + boff[b];
        const int pi = lane < bs ? perm[b0 + lane] : 0;
        T y = spshfl(r, pi);  // (P r)_i = r[perm[i]]
        if (lane >= bs) y = num<T>::zero();
        for (int q = 0; q < bs; ++q) {  // unit lower triangle
            const T yq = spshfl(y, q);
            if (lane > q && lane < bs) y -= F[lane + (size_t)q * bs] * yq;
        }
        for (int q = bs - 1; q >= 0; --q) {  // upper triangle
            if (lane == q) y = spdiv(y, F[q + (size_t)q * bs]);
            const T xq = spshfl(y, q);
            if (lane < q) y -= F[lane + (size_t)q * bs] * xq;
        }
        if (lane < bs) {
            rw[nst + lane] = b0 + lane;
            vl[nst + lane] = y;
        }
        nst += bs;
        t = t2;
    }
    if (over) {
        if (lane == 0) {
            if (!Sri) scnt[c] = 0;
            atomicOr(bad, 2);
        }
        return;
    }
    __syncthreads();
    const int cnt = drop_staged(rw, vl, nst, tau, p, lane, Sri ? Sri + Scp[c] : nullptr,
                                Sri ? Sval + Scp[c] : nullptr);
    if (!Sri && lane == 0) scnt[c] = cnt;
}

// Level expansion for the columns cols[0 .. ncols) (all columns when cols is
// null); column i of S at Scp[i] .. Scp[i] + scnt[i].  Count pass (Jri
// null): cnt[j] = |pattern of s_j| after the removal; fill pass: the
// ascending rows at Jri[Jcp[j] ..].  rb (null for the diagonal V_0): per
// column j its block [rb[2j], rb[2j+1]), whose rows other than j are
// removed.  A column whose t exceeds TC distinct rows or whose s exceeds SC
// rows is appended to over[] (when given) and left alone.
template <class T, int TC, int SC>
__global__ __launch_bounds__(64) void sp_expand_kernel(int n, const int32_t* Scp,
                                                       const int32_t* Sri, const T* Sval,
                                                       const int32_t* scnt, int k, double tau,
                                                       int p, const int32_t* rb,
                                                       const int32_t* cols, int32_t* cnt,
                                                       const int32_t* Jcp, int32_t* Jri,
                                                       int32_t* over, int32_t* nover)
{
    constexpr int HC = 2 * TC;  // accumulator slots
    constexpr int SH = 2 * SC;  // pattern-set slots
    extern __shared__ __align__(16) unsigned char lds[];
    T* hval = (T*)lds;                       // HC
    T* tval = hval + HC;                     // TC
    int32_t* hkey = (int32_t*)(tval + TC);   // HC
    int32_t* hslot = hkey + HC;              // TC: slots in insertion order, later keep flags
    int32_t* trow = hslot + TC;              // TC
    int32_t* skey = trow + TC;               // SH
    int32_t* slist = skey + SH;              // SC
    __shared__ int32_t s_hc, s_sc, s_over;
    const int j = cols ? cols[blockIdx.x] : (int)blockIdx.x;
    const int lane = threadIdx.x;
    (void)n;

    for (int e = lane; e < HC; e += 64) hkey[e] = -1;
    for (int e = lane; e < SH; e += 64) skey[e] = -1;
    if (lane == 0) {
        s_hc = 0;
        s_over = 0;
        trow[0] = j;
        tval[0] = num<T>::one();
        s_sc = 1;
        slist[0] = j;
    }
    __syncthreads();
    if (lane == 0) {
        bool ins;
        hash_slot<SH>(skey, j, ins);
    }
    int tlen = 1;
    __syncthreads();

    for (int lev = 0; lev < k && tlen > 0; ++lev) {
        // t <- S t: sources in ascending row, one column of S at a time
        for (int q = 0; q < tlen; ++q) {
            const int i = trow[q];
            const T ti = tval[q];
            const int b = Scp[i], m = scnt[i];
            for (int e = lane; e < m; e += 64) {
                const int r = Sri[b + e];
                const T prod = mul_rn(Sval[b + e], ti);
                bool ins;
                const int slot = hash_slot<HC>(hkey, r, ins);
                if (slot < 0) {
                    s_over = 1;
                } else if (ins) {
                    const int pos = atomicAdd(&s_hc, 1);
                    if (pos < TC)
                        hslot[pos] = slot;
                    else
                        s_over = 1;
                    hval[slot] = prod;
                } else {
                    hval[slot] = add_rn(hval[slot], prod);
                }
            }
            __syncthreads();
            if (s_over) break;
        }
        if (s_over) break;
        // rank the accumulated rows into ascending order (rows are distinct)
        const int hc = s_hc;
        for (int e = lane; e < hc; e += 64) {
            const int slot = hslot[e];
            const int r = hkey[slot];
            int rank = 0;
            for (int f = 0; f < hc; ++f) rank += hkey[hslot[f]] < r;
            trow[rank] = r;
            tval[rank] = hval[slot];
        }
        __syncthreads();
        for (int e = lane; e < hc; e += 64) hkey[hslot[e]] = -1;
        if (lane == 0) s_hc = 0;
        __syncthreads();
        // dropping by tolerance and count; row j is exempt
        double mx = 0.0;
        for (int e = lane; e < hc; e += 64) mx = fmax(mx, sqm(tval[e]));
        mx = wave_max(mx);
        const double thr = tau > 0.0 ? __dmul_rn(__dmul_rn(tau, tau), mx) : 0.0;
        int ncand = 0;
        for (int e = lane; e < hc; e += 64)
            ncand += trow[e] != j && (tau <= 0.0 || sqm(tval[e]) >= thr);
        ncand = wave_sum(ncand);
        const bool by_count = p > 0 && ncand > p;
        for (int e = lane; e < hc; e += 64) {
            const int r = trow[e];
            const double mg = sqm(tval[e]);
            bool keep = r != j && (tau <= 0.0 || mg >= thr);
            if (keep && by_count) {
                int rank = 0;
                for (int f = 0; f < hc; ++f) {
                    const int rf = trow[f];
                    if (rf == j) continue;
                    const double mf = sqm(tval[f]);
                    if (tau > 0.0 && mf < thr) continue;
                    rank += mf > mg || (mf == mg && rf < r);
                }
                keep = rank < p;
            }
            hslot[e] = keep || r == j;
        }
        __syncthreads();
        // compact in place (a kept entry moves to a position at or below its own)
        int base = 0;
        for (int e0 = 0; e0 < hc; e0 += 64) {
            const int e = e0 + lane;
            const bool keep = e < hc && hslot[e];
            const int r = keep ? trow[e] : 0;
            const T v = keep ? tval[e] : num<T>::zero();
            const uint64_t bal = __ballot(keep);
            __syncthreads();
            if (keep) {
                const int pos = base + __popcll(bal & lanes_below(lane));
                trow[pos] = r;
                tval[pos] = v;
            }
            base += __popcll(bal);
            __syncthreads();
        }
        tlen = base;
        // s_j gains the rows of t
        for (int e = lane; e < tlen; e += 64) {
            bool ins;
            const int slot = hash_slot<SH>(skey, trow[e], ins);
            if (slot < 0) {
                s_over = 1;
            } else if (ins) {
                const int pos = atomicAdd(&s_sc, 1);
                if (pos < SC)
                    slist[pos] = trow[e];
                else
                    s_over = 1;
            }
        }
        __syncthreads();
        if (s_over) break;
    }
    if (s_over) {
        if (lane == 0 && over) over[atomicAdd(nover, 1)] = j;
        return;
    }
    const int sc = s_sc;
    // the final removal: rows of j's block of V_0 other than j
    const int lo = rb ? rb[2 * j] : j, hi = rb ? rb[2 * j + 1] : j + 1;
    if (!Jri) {
        int kept = 0;
        for (int e = lane; e < sc; e += 64) {
            const int r = slist[e];
            kept += r == j || r < lo || r >= hi;
        }
        kept = wave_sum(kept);
        if (lane == 0) cnt[j] = kept;
        return;
    }
    int32_t* dst = Jri + Jcp[j];
    for (int e = lane; e < sc; e += 64) {
        const int r = slist[e];
        if (!(r == j || r < lo || r >= hi)) continue;
        int rank = 0;
        for (int f = 0; f < sc; ++f) {
            const int rf = slist[f];
            rank += rf < r && (rf == j || rf < lo || rf >= hi);
        }
        dst[rank] = r;
    }
}

template <class T>
Err launch_sp_diag(int n, const int32_t* Acp, const int32_t* Ari, const T* Aval, T* d,
                   int32_t* bad, hipStream_t st)
{
    if (n == 0) return {};
    hipLaunchKernelGGL(sp_diag_kernel<T>, dim3((n + 255) / 256), dim3(256), 0, st, n, Acp, Ari,
                       Aval, d, bad);
    DIAF_HIP_TRY(hipGetLastError());
    return {};
}

template <class T>
Err launch_sp_build_s(int n, const int32_t* Acp, const int32_t* Ari, const T* Aval, const T* d,
                      double tau, int p, int32_t* Sri, T* Sval, int32_t* scnt, int32_t* bad,
                      hipStream_t st)
{
    if (n == 0) return {};
    hipLaunchKernelGGL(sp_build_s_kernel<T>, dim3(n), dim3(64), 0, st, n, Acp, Ari, Aval, d, tau,
                       p, Sri, Sval, scnt, bad);
    DIAF_HIP_TRY(hipGetLastError());
    return {};
}

template <class T>
Err launch_sp_block_d(int n, const int32_t* Acp, const int32_t* Ari, const T* Aval,
                      const int32_t* rb, int32_t* cnt, const int32_t* Dcp, int32_t* Dri, T* Dval,
                      hipStream_t st)
{
    if (n == 0) return {};
    hipLaunchKernelGGL(sp_block_d_kernel<T>, dim3((n + 255) / 256), dim3(256), 0, st, n, Acp, Ari,
                       Aval, rb, cnt, Dcp, Dri, Dval);
    DIAF_HIP_TRY(hipGetLastError());
    return {};
}

template <class T>
Err launch_sp_build_s_block(int n, const int32_t* Acp, const int32_t* Ari, const T* Aval,
                            const int32_t* rb, const int32_t* bid, const int32_t* bstart,
                            const int64_t* boff, const T* LU, const int32_t* perm, double tau,
                            int p, int32_t* scnt, const int32_t* Scp, int32_t* Sri, T* Sval,
                            int32_t* bad, hipStream_t st)
{
    if (n == 0) return {};
    hipLaunchKernelGGL(sp_build_s_block_kernel<T>, dim3(n), dim3(64), 0, st, n, Acp, Ari, Aval,
                       rb, bid, bstart, boff, LU, perm, tau, p, scnt, Scp, Sri, Sval, bad);
    DIAF_HIP_TRY(hipGetLastError());
    return {};
}

template <class T, int TC, int SC>
static Err launch_expand_sized(int n, const int32_t* Scp, const int32_t* Sri, const T* Sval,
                               const int32_t* scnt, int k, double tau, int p, const int32_t* rb,
                               const int32_t* cols, int ncols, int32_t* cnt, const int32_t* Jcp,
                               int32_t* Jri, int32_t* over, int32_t* nover, hipStream_t st)
{
    const size_t lds = (size_t)(2 * TC + TC) * sizeof(T) +
                       (size_t)(2 * TC + TC + TC + 2 * SC + SC) * sizeof(int32_t);
    auto kern = sp_expand_kernel<T, TC, SC>;
    DIAF_HIP_TRY(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds));
    hipLaunchKernelGGL(kern, dim3(ncols), dim3(64), lds, st, n, Scp, Sri, Sval, scnt, k, tau, p,
                       rb, cols, cnt, Jcp, Jri, over, nover);
    DIAF_HIP_TRY(hipGetLastError());
    return {};
}

template <class T>
Err launch_sp_expand(int n, const int32_t* Scp, const int32_t* Sri, const T* Sval,
                     const int32_t* scnt, int k, double tau, int p, const int32_t* rb,
                     const int32_t* cols, int ncols, int large, int32_t* cnt, const int32_t* Jcp,
                     int32_t* Jri, int32_t* over, int32_t* nover, hipStream_t st)
{
    if (ncols == 0) return {};
    if (large)
        return launch_expand_sized<T, SpCaps<T>::TL, SpCaps<T>::SL>(
            n, Scp, Sri, Sval, scnt, k, tau, p, rb, cols, ncols, cnt, Jcp, Jri, over, nover, st);
    return launch_expand_sized<T, SP_TC_SMALL, SP_SC_SMALL>(n, Scp, Sri, Sval, scnt, k, tau, p,
                                                            rb, cols, ncols, cnt, Jcp, Jri, over,
                                                            nover, st);
}

#define DIAF_SP_INST(T)                                                                          \
    template Err launch_sp_diag<T>(int, const int32_t*, const int32_t*, const T*, T*, int32_t*,   \
                                   hipStream_t);                                                 \
    template Err launch_sp_build_s<T>(int, const int32_t*, const int32_t*, const T*, const T*,    \
                                      double, int, int32_t*, T*, int32_t*, int32_t*,             \
                                      hipStream_t);                                              \
    template Err launch_sp_block_d<T>(int, const int32_t*, const int32_t*, const T*,             \
                                      const int32_t*, int32_t*, const int32_t*, int32_t*, T*,    \
                                      hipStream_t);                                              \
    template Err launch_sp_build_s_block<T>(int, const int32_t*, const int32_t*, const T*,       \
                                            const int32_t*, const int32_t*, const int32_t*,      \
                                            const int64_t*, const T*, const int32_t*, double,    \
                                            int, int32_t*, const int32_t*, int32_t*, T*,         \
                                            int32_t*, hipStream_t);                              \
    template Err launch_sp_expand<T>(int, const int32_t*, const int32_t*, const T*,              \
                                     const int32_t*, int, double, int, const int32_t*,           \
                                     const int32_t*, int, int, int32_t*, const int32_t*,         \
                                     int32_t*, int32_t*, int32_t*, hipStream_t);
DIAF_SP_INST(double)
DIAF_SP_INST(zc)
#undef DIAF_SP_INST

}  // namespace diaf
