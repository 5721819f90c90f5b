// W pattern by sparsified powers (paper Section 4, Algorithm 1) with V_0 the
// diagonal matrices, for real A.
//
// With V_0 = diag(A) the splitting A = V_0 (I - S) gives S = D^{-1}(A - D):
// S(i, c) = a_ic / a_ii off the diagonal, zero on it.  The columns of S are
// sparsified once (tolerance tau_i relative to the column's largest entry,
// then at most p_i entries, the largest); then, for every column j, t = e_j
// is multiplied by S k times, each product sparsified by (tau_l, p_l) with
// row j exempt, and the pattern of w_j is the union of e_j and every kept t
// (the truncated series I + S + ... + S^k taken entry by entry).  With a
// diagonal V_0 the algorithm's final removal of V_0 minus the identity
// removes nothing.
//
// Reading of the dropping rules (the paper fixes neither the norm nor the
// tie order): magnitudes are compared as squares v*v, the tolerance test
// is v*v >= (tau*tau) * max v*v over the vector (row j included for t),
// a zero parameter disables its rule, and among entries of equal magnitude
// the count rule keeps the lower rows.  Products are formed and summed per
// output row in ascending source row with explicit round-to-nearest
// multiplies and adds, so every value, and hence every dropping decision,
// is reproducible bit for bit.
//
// Kernels: a diagonal gather; one wave per column of S for the scaling and
// the initial dropping (entries staged in LDS); one wave per column j for
// the level expansion.  The expansion walks the sources of t in ascending
// row, one after the other; the entries of one column of S go to the 64
// lanes, whose rows are distinct, into an LDS hash accumulator (row ->
// slot, insertion by compare-and-swap), so per output row the partial sums
// arrive in source order.  The accumulated rows are then ranked into
// ascending order, dropped and compacted in place, and added to an LDS hash
// set that holds the pattern of s_j.  Two LDS sizes are built; columns that
// outgrow the smaller one are listed and rerun with the larger one.
#include "dcommon.h"
#include "factor_kernels.h"

namespace diaf {

namespace {

constexpr int SB_CAP = 1024;  // entries of one column of A held in LDS by the S build

__device__ inline double sqm(double v) { return __dmul_rn(v, v); }

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

}  // namespace

// d[c] = a_cc (columns of A have their diagonal; validated before).  Bit 0
// of *bad is set for a zero diagonal.
__global__ void sp_diag_kernel(int n, const int32_t* Acp, const int32_t* Ari, const double* Aval,
                               double* d, int32_t* bad)
{
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    double v = 0.0;
    for (int q = Acp[c]; q < Acp[c + 1]; ++q)
        if (Ari[q] == c) {
            v = Aval[q];
            break;
        }
    d[c] = v;
    if (v == 0.0) atomicOr(bad, 1);
}

// Column c of S, sparsified by (tau, p), written at Acp[c] .. Acp[c] +
// scnt[c] of Sri/Sval with ascending rows.  Bit 1 of *bad is set for a
// column of A longer than SB_CAP.
__global__ __launch_bounds__(64) void sp_build_s_kernel(int n, const int32_t* Acp,
                                                        const int32_t* Ari, const double* Aval,
                                                        const double* d, double tau, int p,
                                                        int32_t* Sri, double* Sval, int32_t* scnt,
                                                        int32_t* bad)
{
    __shared__ int32_t rw[SB_CAP];
    __shared__ double vl[SB_CAP];
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
    double mx = 0.0;
    for (int q = lane; q < na; q += 64) {
        const int i = Ari[a0 + q];
        double v = 0.0;
        if (i != c) {
            v = __ddiv_rn(Aval[a0 + q], d[i]);
            mx = fmax(mx, sqm(v));
        }
        rw[q] = i == c ? -1 : i;  // the diagonal of A is not an entry of S
        vl[q] = v;
    }
    mx = wave_max(mx);
    const double thr = tau > 0.0 ? __dmul_rn(__dmul_rn(tau, tau), mx) : 0.0;
    __syncthreads();
    int ncand = 0;
    for (int q = lane; q < na; q += 64)
        ncand += rw[q] >= 0 && (tau <= 0.0 || sqm(vl[q]) >= thr);
    ncand = wave_sum(ncand);
    const bool by_count = p > 0 && ncand > p;
    int base = 0;
    for (int q0 = 0; q0 < na; q0 += 64) {
        const int q = q0 + lane;
        bool keep = false;
        int row = -1;
        double v = 0.0;
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
        if (keep) {
            const int pos = base + __popcll(bal & lanes_below(lane));
            Sri[a0 + pos] = row;
            Sval[a0 + pos] = v;
        }
        base += __popcll(bal);
    }
    if (lane == 0) scnt[c] = base;
}

// Level expansion for the columns cols[0 .. ncols) (all columns when cols is
// null).  Count pass (Jri null): cnt[j] = |pattern of s_j|.  Fill pass: the
// ascending rows at Jri[Jcp[j] ..].  A column whose t exceeds TC distinct
// rows or whose s exceeds SC rows is appended to over[] (when given) and
// left alone.
template <int TC, int SC>
__global__ __launch_bounds__(64) void sp_expand_kernel(int n, const int32_t* Acp,
                                                       const int32_t* Sri, const double* Sval,
                                                       const int32_t* scnt, int k, double tau,
                                                       int p, const int32_t* cols, int32_t* cnt,
                                                       const int32_t* Jcp, int32_t* Jri,
                                                       int32_t* over, int32_t* nover)
{
    constexpr int HC = 2 * TC;  // accumulator slots
    constexpr int SH = 2 * SC;  // pattern-set slots
    extern __shared__ __align__(16) unsigned char lds[];
    double* hval = (double*)lds;             // HC
    double* tval = hval + HC;                // TC
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
        tval[0] = 1.0;
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
            const double ti = tval[q];
            const int b = Acp[i], m = scnt[i];
            for (int e = lane; e < m; e += 64) {
                const int r = Sri[b + e];
                const double prod = __dmul_rn(Sval[b + e], ti);
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
                    hval[slot] = __dadd_rn(hval[slot], prod);
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
            const double v = keep ? tval[e] : 0.0;
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
    if (!Jri) {
        if (lane == 0) cnt[j] = sc;
        return;
    }
    int32_t* dst = Jri + Jcp[j];
    for (int e = lane; e < sc; e += 64) {
        const int r = slist[e];
        int rank = 0;
        for (int f = 0; f < sc; ++f) rank += slist[f] < r;
        dst[rank] = r;
    }
}

Err launch_sp_diag(int n, const int32_t* Acp, const int32_t* Ari, const double* Aval, double* d,
                   int32_t* bad, hipStream_t st)
{
    if (n == 0) return {};
    hipLaunchKernelGGL(sp_diag_kernel, dim3((n + 255) / 256), dim3(256), 0, st, n, Acp, Ari, Aval,
                       d, bad);
    DIAF_HIP_TRY(hipGetLastError());
    return {};
}

Err launch_sp_build_s(int n, const int32_t* Acp, const int32_t* Ari, const double* Aval,
                      const double* d, double tau, int p, int32_t* Sri, double* Sval,
                      int32_t* scnt, int32_t* bad, hipStream_t st)
{
    if (n == 0) return {};
    hipLaunchKernelGGL(sp_build_s_kernel, dim3(n), dim3(64), 0, st, n, Acp, Ari, Aval, d, tau, p,
                       Sri, Sval, scnt, bad);
    DIAF_HIP_TRY(hipGetLastError());
    return {};
}

template <int TC, int SC>
static Err launch_expand_sized(int n, const int32_t* Acp, const int32_t* Sri, const double* Sval,
                               const int32_t* scnt, int k, double tau, int p, const int32_t* cols,
                               int ncols, int32_t* cnt, const int32_t* Jcp, int32_t* Jri,
                               int32_t* over, int32_t* nover, hipStream_t st)
{
    const size_t lds = (size_t)(2 * TC + TC) * sizeof(double) +
                       (size_t)(2 * TC + TC + TC + 2 * SC + SC) * sizeof(int32_t);
    auto kern = sp_expand_kernel<TC, SC>;
    DIAF_HIP_TRY(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds));
    hipLaunchKernelGGL(kern, dim3(ncols), dim3(64), lds, st, n, Acp, Sri, Sval, scnt, k, tau, p,
                       cols, cnt, Jcp, Jri, over, nover);
    DIAF_HIP_TRY(hipGetLastError());
    return {};
}

Err launch_sp_expand(int n, const int32_t* Acp, const int32_t* Sri, const double* Sval,
                     const int32_t* scnt, int k, double tau, int p, const int32_t* cols, int ncols,
                     int large, int32_t* cnt, const int32_t* Jcp, int32_t* Jri, int32_t* over,
                     int32_t* nover, hipStream_t st)
{
    if (ncols == 0) return {};
    if (large)
        return launch_expand_sized<SP_TC_LARGE, SP_SC_LARGE>(n, Acp, Sri, Sval, scnt, k, tau, p,
                                                             cols, ncols, cnt, Jcp, Jri, over,
                                                             nover, st);
    return launch_expand_sized<SP_TC_SMALL, SP_SC_SMALL>(n, Acp, Sri, Sval, scnt, k, tau, p, cols,
                                                         ncols, cnt, Jcp, Jri, over, nover, st);
}

}  // namespace diaf
