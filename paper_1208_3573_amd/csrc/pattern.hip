// W-pattern construction (paper Section 4).
//
// pattern(A^2) is the truncated Neumann series W = I + S + S^2 pattern of
// Section 4.1 with V_0 = diagonals, truncation 2 and no dropping, taken
// symbolically: column j is the union of the row sets of A(:, c) over
// c in rows(A(:, j)).  The 1-hop top-p pattern keeps pattern(A) and adds the
// p two-hop rows i with the largest |A|^2 path weight sum_c |a_ic||a_cj|
// (numerical dropping by count, Section 4.1); products are formed and
// summed in ascending c with explicit round-to-nearest operations so the
// scores are reproducible bit for bit, ties going to the lower row.
//
// Each column is one workgroup: candidates are gathered into LDS as one
// sorted run per inner column, merged pairwise (ceil(log2) rounds of one
// binary search per entry) and deduplicated.  A first launch counts, a
// second fills the rows at the scanned offsets.
#include <hipcub/hipcub.hpp>

#include "dcommon.h"
#include "factor_kernels.h"

namespace diaf {

// Candidates of column j of a union pattern: the total length of the inner
// lists (Icp/Iri) named by the outer list of column j (Ocp/Ori).
__global__ void cand_count_kernel(int n, const int32_t* Ocp, const int32_t* Ori,
                                  const int32_t* Icp, int32_t* cnt, int32_t* maxcnt)
{
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    int s = 0;
    if (j < n) {
        for (int p = Ocp[j]; p < Ocp[j + 1]; ++p) {
            int c = Ori[p];
            s += Icp[c + 1] - Icp[c];
        }
        cnt[j] = s;
    }
    // wave max then one atomic per wave
    for (int o = 32; o > 0; o >>= 1) s = max(s, __shfl_xor(s, o));
    if ((threadIdx.x & 63) == 0) atomicMax(maxcnt, s);
}

Err launch_cand_count(int n, const int32_t* Ocp, const int32_t* Ori, const int32_t* Icp,
                      int32_t* cnt, int32_t* maxcnt_dev, hipStream_t st)
{
    hipLaunchKernelGGL(cand_count_kernel, dim3((n + 255) / 256), dim3(256), 0, st, n, Ocp, Ori, Icp,
                       cnt, maxcnt_dev);
    DIAF_HIP_TRY(hipGetLastError());
    return {};
}

__global__ void column_sizes_kernel(int n, const int32_t* Acp, const int32_t* Jcp,
                                    const int32_t* Jri, int32_t* kout, int32_t* tout)
{
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    int k = Jcp[j + 1] - Jcp[j];
    int t = 0;
    for (int a = 0; a < k; ++a) {
        int c = Jri[Jcp[j] + a];
        t += Acp[c + 1] - Acp[c];
    }
    kout[j] = k;
    tout[j] = t;
}

Err launch_column_sizes(int n, const int32_t* Acp, const int32_t* Jcp, const int32_t* Jri,
                        int32_t* kout, int32_t* tout, hipStream_t st)
{
    hipLaunchKernelGGL(column_sizes_kernel, dim3((n + 255) / 256), dim3(256), 0, st, n, Acp, Jcp,
                       Jri, kout, tout);
    DIAF_HIP_TRY(hipGetLastError());
    return {};
}

// Factor launch classes.  Column sel[i] (i when sel is null) goes to the
// first class c with k <= kcap[c] and t <= tcap[c], ncls when none fits;
// key/val receive (class, column) for a stable sort by class, counts[c] the
// number of columns of class c, and maxes[0..1] the largest k and t over all
// n columns (maxes null: not taken).  Per-workgroup tallies in LDS, one
// global atomic per workgroup and class.
__global__ void __launch_bounds__(256) classify_kernel(int n, int m, const int32_t* sel,
                                                       const int32_t* kk, const int32_t* tt,
                                                       ColumnClasses cc, int32_t* key,
                                                       int32_t* val, int32_t* counts,
                                                       int32_t* maxes)
{
    __shared__ int32_t tally[ColumnClasses::kMax + 1];
    __shared__ int32_t mx[2];
    const int tid = threadIdx.x;
    if (tid <= cc.ncls) tally[tid] = 0;
    if (tid < 2) mx[tid] = 0;
    __syncthreads();
    const int i = blockIdx.x * blockDim.x + tid;
    if (i < m) {
        const int j = sel ? sel[i] : i;
        const int k = kk[j], t = tt[j];
        int c = 0;
        while (c < cc.ncls && !(k <= cc.kcap[c] && t <= cc.tcap[c])) ++c;
        key[i] = c;
        val[i] = j;
        atomicAdd(&tally[c], 1);
    }
    if (maxes) {
        int km = 0, tm = 0;
        if (i < n) { km = kk[i]; tm = tt[i]; }
        for (int o = 32; o > 0; o >>= 1) {
            km = max(km, __shfl_xor(km, o));
            tm = max(tm, __shfl_xor(tm, o));
        }
        if ((tid & 63) == 0) {
            atomicMax(&mx[0], km);
            atomicMax(&mx[1], tm);
        }
    }
    __syncthreads();
    if (tid <= cc.ncls && tally[tid]) atomicAdd(&counts[tid], tally[tid]);
    if (maxes && tid < 2 && mx[tid]) atomicMax(&maxes[tid], mx[tid]);
}

Err launch_classify_columns(int n, int m, const int32_t* sel, const int32_t* kk, const int32_t* tt,
                            const ColumnClasses& cc, int32_t* sorted, int32_t* counts,
                            int32_t* maxes, hipStream_t st)
{
    if (cc.ncls < 1 || cc.ncls > ColumnClasses::kMax) return {DIAF_EINVAL, "internal: column classes out of range"};
    DIAF_HIP_TRY(hipMemsetAsync(counts, 0, sizeof(int32_t) * (cc.ncls + 1), st));
    if (maxes) DIAF_HIP_TRY(hipMemsetAsync(maxes, 0, sizeof(int32_t) * 2, st));
    const int cover = maxes ? std::max(n, m) : m;
    if (cover == 0) return {};
    int32_t *key = nullptr, *kout = nullptr, *val = nullptr;
    const size_t mm = (size_t)std::max(m, 1);
    DIAF_TRY(amalloc((void**)&key, sizeof(int32_t) * mm, st));
    DIAF_TRY(amalloc((void**)&kout, sizeof(int32_t) * mm, st));
    DIAF_TRY(amalloc((void**)&val, sizeof(int32_t) * mm, st));
    hipLaunchKernelGGL(classify_kernel, dim3((unsigned)((cover + 255) / 256)), dim3(256), 0, st, n,
                       m, sel, kk, tt, cc, key, val, counts, maxes);
    DIAF_HIP_TRY(hipGetLastError());
    if (m > 0) {
        int bits = 1;
        while ((1 << bits) <= cc.ncls) ++bits;
        size_t tmp_bytes = 0;
        DIAF_HIP_TRY(hipcub::DeviceRadixSort::SortPairs(nullptr, tmp_bytes, key, kout, val, sorted,
                                                        m, 0, bits, st));
        void* tmp = nullptr;
        DIAF_TRY(amalloc(&tmp, tmp_bytes, st));
        DIAF_HIP_TRY(hipcub::DeviceRadixSort::SortPairs(tmp, tmp_bytes, key, kout, val, sorted, m,
                                                        0, bits, st));
        afree(tmp, st);
    }
    afree(key, st);
    afree(kout, st);
    afree(val, st);
    return {};
}

// Ascending sort of m column indices (values below n).
Err sort_columns(int n, int m, const int32_t* in, int32_t* out, hipStream_t st)
{
    if (m == 0) return {};
    int bits = 1;
    while ((1ll << bits) < (int64_t)n) ++bits;
    size_t tmp_bytes = 0;
    DIAF_HIP_TRY(hipcub::DeviceRadixSort::SortKeys(nullptr, tmp_bytes, in, out, m, 0, bits, st));
    void* tmp = nullptr;
    DIAF_TRY(amalloc(&tmp, tmp_bytes, st));
    DIAF_HIP_TRY(hipcub::DeviceRadixSort::SortKeys(tmp, tmp_bytes, in, out, m, 0, bits, st));
    afree(tmp, st);
    return {};
}

// Inclusive sum of x over the lanes of the wave up to this one.
__device__ inline int wave_incl_scan(int x)
{
    const int lane = threadIdx.x & 63;
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    return x;
}

// Block-wide exclusive scan of 0/1 flags in place (returns total).  Each
// thread owns a contiguous chunk; chunk sums are scanned by wave shuffles
// and across waves through red (at least blockDim.x / 64 ints).
__device__ inline int block_scan01(int32_t* f, int cnt, int32_t* red)
{
    const int nt = blockDim.x, tid = threadIdx.x;
    const int chunk = (cnt + nt - 1) / nt;
    const int b = tid * chunk, e = min(cnt, b + chunk);
    int s = 0;
    for (int i = b; i < e; ++i) s += f[i];
    const int x = wave_incl_scan(s);
    const int wv = tid >> 6;
    if ((tid & 63) == 63 || tid == nt - 1) red[wv] = x;
    __syncthreads();
    int before = 0, tot = 0;
    for (int w = 0; w < (nt + 63) >> 6; ++w) {
        const int t = red[w];
        before += w < wv ? t : 0;
        tot += t;
    }
    int run = before + x - s;
    for (int i = b; i < e; ++i) { const int v = f[i]; f[i] = run; run += v; }
    __syncthreads();
    return tot;
}

// The q-th largest (1-based, q <= cnt) of the non-negative doubles
// v[0..cnt), by radix selection on their bit patterns (which order as the
// values): up to 8 passes over 8-bit digits from the top, each counting the
// values that match the digits fixed so far into 256 bins (hist) and fixing
// the digit in which the q-th falls.  Once that bin holds exactly as many
// values as the rank still needed, the q-th is their minimum, taken in one
// more sweep (usually after a few passes).  pick holds 3 ints; blockDim.x is
// a multiple of 64.
__device__ inline double block_kth_largest(const double* v, int cnt, int q, int32_t* hist,
                                           int32_t* pick)
{
    const int tid = threadIdx.x, nt = blockDim.x;
    uint64_t prefix = 0, mask = 0;
    int rem = q;
    for (int shift = 56; shift >= 0; shift -= 8) {
        for (int b = tid; b < 256; b += nt) hist[b] = 0;
        __syncthreads();
        for (int t = tid; t < cnt; t += nt) {
            const uint64_t key = (uint64_t)__double_as_longlong(v[t]) & 0x7fffffffffffffffull;
            if ((key & mask) == prefix) atomicAdd(&hist[(key >> shift) & 255], 1);
        }
        __syncthreads();
        if (tid < 64) {
            // lane l holds bins 255 - 4l down to 252 - 4l
            int h[4], loc = 0;
            for (int r = 0; r < 4; ++r) { h[r] = hist[255 - 4 * tid - r]; loc += h[r]; }
            const int x = wave_incl_scan(loc), excl = x - loc;
            if (excl < rem && rem <= x) {
                int run = excl, r = 0;
                while (r < 3 && run + h[r] < rem) { run += h[r]; ++r; }
                pick[0] = 255 - 4 * tid - r;
                pick[1] = rem - run;
                pick[2] = h[r];
            }
        }
        __syncthreads();
        prefix |= (uint64_t)(uint32_t)pick[0] << shift;
        mask |= 255ull << shift;
        rem = pick[1];
        if (shift > 0 && pick[2] == rem) {
            // every value in the bin ranks at or above the q-th: its minimum
            uint64_t lo = ~0ull;
            for (int t = tid; t < cnt; t += nt) {
                const uint64_t key = (uint64_t)__double_as_longlong(v[t]) & 0x7fffffffffffffffull;
                if ((key & mask) == prefix) lo = key < lo ? key : lo;
            }
            for (int o = 32; o > 0; o >>= 1) {
                const uint64_t y = __shfl_xor(lo, o);
                lo = y < lo ? y : lo;
            }
            // wave minima through hist (read by wave 0 before the barrier
            // above), as 32-bit halves
            const int w0 = tid >> 6;
            if ((tid & 63) == 0) {
                hist[2 * w0] = (int32_t)(uint32_t)lo;
                hist[2 * w0 + 1] = (int32_t)(uint32_t)(lo >> 32);
            }
            __syncthreads();
            for (int w = 0; w < (nt >> 6); ++w) {
                const uint64_t y = (uint64_t)(uint32_t)hist[2 * w] |
                                   ((uint64_t)(uint32_t)hist[2 * w + 1] << 32);
                lo = y < lo ? y : lo;
            }
            __syncthreads();  // hist is reused by the caller's next call
            return __longlong_as_double((long long)lo);
        }
    }
    return __longlong_as_double((long long)prefix);
}

// pattern(A^2), one block per column; cap candidates max (power of two),
// dynamic LDS: keys[cap] u32, off[cap+1] i32, red[nthreads+1] i32,
// keys2[cap] u32.
// Column j of the union pattern: the sorted union of the inner lists
// (Icp/Iri) named by the outer list of column j (Ocp/Ori).  pattern(A^2):
// outer and inner lists are both the columns of A.  The gathered inner
// lists are na sorted runs, merged pairwise in ceil(log2 na) rounds (equal
// rows: the left group's first), then duplicates dropped.
__global__ void pattern_a2_kernel(int n, const int32_t* Ocp, const int32_t* Ori,
                                  const int32_t* Icp, const int32_t* Iri, int cap, int32_t* cnt,
                                  const int32_t* Jcp, int32_t* Jri)
{
    extern __shared__ __align__(16) unsigned char lds[];
    uint32_t* keys = (uint32_t*)lds;
    int32_t* off = (int32_t*)(keys + cap);
    int32_t* red = off + cap + 1;
    uint32_t* keys2 = (uint32_t*)(red + blockDim.x + 1);
    __shared__ int32_t s_tot;
    const int j = blockIdx.x;
    const int tid = threadIdx.x;
    const int a0 = Ocp[j], na = Ocp[j + 1] - a0;
    if (tid == 0) {
        off[0] = 0;
        for (int q = 0; q < na; ++q) {
            int c = Ori[a0 + q];
            off[q + 1] = off[q] + (Icp[c + 1] - Icp[c]);
        }
        s_tot = off[na];
    }
    __syncthreads();
    const int T = s_tot;
    // the gather writes into the buffer that the last round leaves in keys
    int rounds = 0;
    while ((1 << rounds) < na) ++rounds;
    uint32_t* gbuf = (rounds & 1) ? keys2 : keys;
    // run containing gather position t: the last q < na with off[q] <= t
    // (inner lists may be empty)
    auto run_of = [&](int t) {
        int lo = 0, hi = na - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (off[mid] <= t) lo = mid; else hi = mid - 1;
        }
        return lo;
    };
    for (int t = tid; t < T; t += blockDim.x) {
        const int q = run_of(t);
        const int c = Ori[a0 + q];
        gbuf[t] = (uint32_t)Iri[Icp[c] + (t - off[q])];
    }
    __syncthreads();
    for (int r = 0; r < rounds; ++r) {
        const uint32_t* src = ((rounds - r) & 1) ? keys2 : keys;
        uint32_t* dst = ((rounds - r) & 1) ? keys : keys2;
        for (int t = tid; t < T; t += blockDim.x) {
            // merged groups of 2^r runs cover contiguous gather ranges, so
            // the run at position t names the group of the entry there
            const uint32_t key = src[t];
            const int g = run_of(t) >> r, h = g ^ 1;
            const int gs = off[g << r];
            if ((h << r) >= na) {
                dst[t] = key;
                continue;
            }
            const int hs = off[h << r], he = off[min((h + 1) << r, na)];
            int lo = hs, hi = he;  // partner entries below (left) or not above (right)
            if (g < h) {
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    if (src[mid] < key) lo = mid + 1; else hi = mid;
                }
            } else {
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    if (src[mid] <= key) lo = mid + 1; else hi = mid;
                }
            }
            dst[min(gs, hs) + (t - gs) + (lo - hs)] = key;
        }
        __syncthreads();
    }
    // unique flags into off[] (reused)
    for (int t = tid; t < T; t += blockDim.x) off[t] = (t == 0 || keys[t] != keys[t - 1]) ? 1 : 0;
    __syncthreads();
    int m = block_scan01(off, T, red);
    if (!Jri) {
        if (tid == 0) cnt[j] = m;
        return;
    }
    int32_t* out = Jri + Jcp[j];
    for (int t = tid; t < T; t += blockDim.x)
        if (t == 0 || keys[t] != keys[t - 1]) out[off[t]] = (int32_t)keys[t];
}

// Pattern of the initial subspace V_0 of Algorithm 2: the diagonal
// (v0 = 0) or the Gauss-Seidel structure (Definition 4.1): the diagonal plus
// the strictly upper (v0 = 1) or lower (v0 = 2) part of pattern(A), column
// by column.  Counting pass (rows == nullptr) or filling pass.
__global__ void v0_pattern_kernel(int n, const int32_t* Acp, const int32_t* Ari, int v0,
                                  int32_t* cnt, const int32_t* Vcp, int32_t* Vri)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    int c = 0;
    for (int p = Acp[j]; p < Acp[j + 1]; ++p) {
        const int i = Ari[p];
        const bool keep = i == j || (v0 == 1 && i < j) || (v0 == 2 && i > j);
        if (!keep) continue;
        if (Vri) Vri[Vcp[j] + c] = i;
        ++c;
    }
    if (!Vri) cnt[j] = c;
}

Err launch_v0_pattern(int n, const int32_t* Acp, const int32_t* Ari, int v0, int32_t* cnt,
                      const int32_t* Vcp, int32_t* Vri, hipStream_t st)
{
    if (n == 0) return {};
    hipLaunchKernelGGL(v0_pattern_kernel, dim3((n + 255) / 256), dim3(256), 0, st, n, Acp, Ari, v0,
                       cnt, Vcp, Vri);
    DIAF_HIP_TRY(hipGetLastError());
    return {};
}

static int pow2_at_least(int x)
{
    int p = 1;
    while (p < x) p <<= 1;
    return p;
}

Err launch_pattern_a2(int n, const int32_t* Ocp, const int32_t* Ori, const int32_t* Icp,
                      const int32_t* Iri, int maxcand, int32_t* cnt, const int32_t* Jcp,
                      int32_t* Jri, hipStream_t st)
{
    if (n == 0) return {};
    int cap = pow2_at_least(maxcand < 64 ? 64 : maxcand);
    if (cap > 8192) return {DIAF_EUNSUPPORTED, "pattern(A^2): more than 8192 candidates in a column"};
    int nt = cap <= 256 ? 64 : (cap <= 4096 ? 256 : 1024);
    size_t lds = 2 * sizeof(uint32_t) * cap + sizeof(int32_t) * (cap + 1) + sizeof(int32_t) * (nt + 1);
    DIAF_HIP_TRY(hipFuncSetAttribute((const void*)pattern_a2_kernel,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(pattern_a2_kernel, dim3(n), dim3(nt), lds, st, n, Ocp, Ori, Icp, Iri, cap,
                       cnt, Jcp, Jri);
    DIAF_HIP_TRY(hipGetLastError());
    return {};
}

// pattern(A) + top-p two-hop rows.  Keys: (row << 32) | (q << 12) | t for the
// entry at gather position t, which comes from the q-th column c of
// pattern(A(:, j)) (t, q < 4096 since cap <= 4096); gather positions follow
// ascending c, so equal rows order by ascending c, and every key is unique.
// The gather is na runs already sorted by row (the rows of each A(:, c)),
// merged pairwise in ceil(log2 na) rounds; a round-r element belongs to the
// merged group q >> r, so it finds its new place by one binary search in the
// partner group.
// Dynamic LDS: keys[cap] u64, prod[cap] f64, sc[cap] f64, off[cap+1] i32,
// scrow[cap] i32, red[nthreads+1] i32, sel[256] i32, cst[cap] i32.
template <class T>
__global__ void pattern_1hop_kernel(int n, const int32_t* Acp, const int32_t* Ari, const T* Aval,
                                    int ptop, int cap, const int32_t* cols, int32_t* cnt,
                                    int32_t* Jtmp)
{
    extern __shared__ __align__(16) unsigned char lds[];
    uint64_t* keys = (uint64_t*)lds;
    double* prod = (double*)(keys + cap);
    double* sc = prod + cap;
    int32_t* off = (int32_t*)(sc + cap);
    int32_t* scrow = off + cap + 1;
    int32_t* red = scrow + cap;
    int32_t* sel = red + blockDim.x + 1;
    int32_t* cst = sel + 256;
    __shared__ int32_t s_nsel, s_above, s_equal, s_pick[3], s_hist[256];
    const int j = cols[blockIdx.x];
    const int tid = threadIdx.x;
    const int a0 = Acp[j], na = Acp[j + 1] - a0;
    // merge rounds; the gather writes into the buffer that the last round
    // leaves in keys, and |A(c, j)| is staged in the other one
    int rounds = 0;
    while ((1 << rounds) < na) ++rounds;
    uint64_t* gbuf = (rounds & 1) ? (uint64_t*)sc : keys;
    double* acj = (rounds & 1) ? (double*)keys : sc;
    // off[q] = total length of A(:, c) over the first q columns c of
    // pattern(A(:, j)) (an exclusive scan), off[na] = the gathered count.
    // Staged in LDS for the gather and the candidate test (the score arrays
    // are free until the scores): the rows c of A(:, j) (ascending) in
    // scrow, |A(c, j)| in acj, the start of A(:, c) in cst.
    for (int q = tid; q < na; q += blockDim.x) {
        const int c = Ari[a0 + q];
        const int c0 = Acp[c];
        off[q] = Acp[c + 1] - c0;
        cst[q] = c0;
        scrow[q] = c;
        if constexpr (num<T>::is_complex) {
            const T y = Aval[a0 + q];
            acj[q] = __dsqrt_rn(__dadd_rn(__dmul_rn(y.x, y.x), __dmul_rn(y.y, y.y)));
        } else {
            acj[q] = fabs(Aval[a0 + q]);
        }
    }
    __syncthreads();
    const int Tn = block_scan01(off, na, red);
    if (tid == 0) off[na] = Tn;
    __syncthreads();
    for (int t = tid; t < Tn; t += blockDim.x) {
        int lo = 0, hi = na - 1;
        while (lo < hi) {
            int mid = (lo + hi + 1) >> 1;
            if (off[mid] <= t) lo = mid; else hi = mid - 1;
        }
        const int p = cst[lo] + (t - off[lo]);
        double aic;
        if constexpr (num<T>::is_complex) {
            const T x = Aval[p];
            aic = __dsqrt_rn(__dadd_rn(__dmul_rn(x.x, x.x), __dmul_rn(x.y, x.y)));
        } else {
            aic = fabs(Aval[p]);
        }
        prod[t] = __dmul_rn(aic, acj[lo]);
        gbuf[t] = ((uint64_t)(uint32_t)Ari[p] << 32) | ((uint32_t)lo << 12) | (uint32_t)t;
    }
    __syncthreads();
    for (int r = 0; r < rounds; ++r) {
        const uint64_t* src = ((rounds - r) & 1) ? (const uint64_t*)sc : keys;
        uint64_t* dst = ((rounds - r) & 1) ? keys : (uint64_t*)sc;
        for (int t = tid; t < Tn; t += blockDim.x) {
            const uint64_t key = src[t];
            const int g = (int)((key >> 12) & 0xfff) >> r, h = g ^ 1;
            const int gs = off[g << r];
            if ((h << r) >= na) {
                dst[t] = key;  // no partner group this round
                continue;
            }
            const int hs = off[h << r], he = off[min((h + 1) << r, na)];
            int lo = hs, hi = he;  // first partner key above this one
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (src[mid] < key) lo = mid + 1; else hi = mid;
            }
            dst[min(gs, hs) + (t - gs) + (lo - hs)] = key;
        }
        __syncthreads();
    }
    // segment starts of rows outside pattern(A(:, j)) are the candidates;
    // the rows of A(:, j) are copied to cst for the final union (scrow is
    // reused for the candidates' rows)
    for (int q = tid; q < na; q += blockDim.x) cst[q] = scrow[q];
    for (int t = tid; t < Tn; t += blockDim.x) {
        int row = (int)(keys[t] >> 32);
        int start = (t == 0 || (keys[t] >> 32) != (keys[t - 1] >> 32));
        int inA = 0;
        if (start) {
            int lo = 0, hi = na - 1;
            while (lo <= hi) {
                int mid = (lo + hi) >> 1;
                int v = scrow[mid];
                if (v == row) { inA = 1; break; }
                if (v < row) lo = mid + 1; else hi = mid - 1;
            }
        }
        off[t] = (start && !inA) ? 1 : 0;
    }
    __syncthreads();
    const int nc = block_scan01(off, Tn, red);
    // score = sequential sum of the segment's products in ascending c
    for (int t = tid; t < Tn; t += blockDim.x) {
        int slot = off[t];
        int isc = (t + 1 < Tn ? off[t + 1] : nc) != slot;
        if (!isc) continue;
        int row = (int)(keys[t] >> 32);
        double s = 0.0;
        for (int u = t; u < Tn && (int)(keys[u] >> 32) == row; ++u)
            s = __dadd_rn(s, prod[keys[u] & 0xfff]);
        sc[slot] = s;
        scrow[slot] = row;
    }
    if (tid == 0) { s_nsel = 0; s_above = 0; s_equal = 0; }
    __syncthreads();
    // top-ptop: larger score first, lower row on ties.  With s* the take-th
    // largest score, every candidate above s* is taken and the rest come
    // from the candidates equal to s* in ascending row (= slot) order.
    const int take = nc < ptop ? nc : ptop;
    if (nc <= ptop) {
        for (int s = tid; s < nc; s += blockDim.x) sel[s] = scrow[s];
    } else {
        const double ss = block_kth_largest(sc, nc, take, s_hist, s_pick);
        for (int s = tid; s < nc; s += blockDim.x) {
            off[s] = sc[s] == ss;
            if (sc[s] > ss) atomicAdd(&s_above, 1);
            if (sc[s] == ss) atomicAdd(&s_equal, 1);
        }
        __syncthreads();
        const int need = take - s_above;
        // rank among the candidates equal to s*, unless all of them are taken
        // (s_equal >= need since s* is the take-th largest)
        const bool all_equal = s_equal == need;
        if (!all_equal) block_scan01(off, nc, red);
        for (int s = tid; s < nc; s += blockDim.x) {
            const double v = sc[s];
            if (v > ss || (v == ss && (all_equal || off[s] < need)))
                sel[atomicAdd(&s_nsel, 1)] = scrow[s];
        }
    }
    __syncthreads();
    // output = sorted(rows(A(:, j)) U sel), into the column's slot of
    // capacity |A(:, j)| + ptop.  The picks are distinct and outside
    // A(:, j), so each entry's place is the number of rows of both sets
    // below it.
    const int tot = na + take;
    if (tid == 0) cnt[j] = tot;
    int32_t* out = Jtmp + a0 + (size_t)j * ptop;
    for (int t = tid; t < na; t += blockDim.x) {
        const int row = cst[t];
        int below = 0;
        for (int u = 0; u < take; ++u) below += sel[u] < row;
        out[t + below] = row;
    }
    for (int u = tid; u < take; u += blockDim.x) {
        const int x = sel[u];
        int lo = 0, hi = na;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (cst[mid] < x) lo = mid + 1; else hi = mid;
        }
        int below = 0;
        for (int v = 0; v < take; ++v) below += sel[v] < x;
        out[lo + below] = x;
    }
}

// Jri[Jcp[j] ..] = the cnt[j] rows of column j's slot in Jtmp (one wave per
// column).
__global__ void compact_slots_kernel(int n, const int32_t* Acp, int ptop, const int32_t* cnt,
                                     const int32_t* Jtmp, const int32_t* Jcp, int32_t* Jri)
{
    const int j = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (j >= n) return;
    const int32_t* src = Jtmp + Acp[j] + (size_t)j * ptop;
    int32_t* dst = Jri + Jcp[j];
    for (int t = lane; t < cnt[j]; t += 64) dst[t] = src[t];
}

Err launch_compact_slots(int n, const int32_t* Acp, int ptop, const int32_t* cnt,
                         const int32_t* Jtmp, const int32_t* Jcp, int32_t* Jri, hipStream_t st)
{
    if (n == 0) return {};
    hipLaunchKernelGGL(compact_slots_kernel, dim3((n + 3) / 4), dim3(256), 0, st, n, Acp, ptop, cnt,
                       Jtmp, Jcp, Jri);
    DIAF_HIP_TRY(hipGetLastError());
    return {};
}

// cols: the columns of one size class, all with at most cand_max two-hop
// candidates; the LDS buffers hold pow2(cand_max + ptop + 1) keys, enough for
// the candidates and for the final merge of pattern(A(:, j)) with the picks.
template <class T>
Err launch_pattern_1hop(int n, const int32_t* Acp, const int32_t* Ari, const T* Aval, int ptop,
                        int cand_max, const int32_t* cols, int ncols, int32_t* cnt,
                        int32_t* Jtmp, hipStream_t st)
{
    if (ncols == 0) return {};
    if (ptop > 256 || ptop < 0) return {DIAF_EUNSUPPORTED, "1-hop pattern: 0..256 extra rows"};
    int cap = pow2_at_least(cand_max + ptop + 1 < 256 ? 256 : cand_max + ptop + 1);
    if (cap > 4096) return {DIAF_EUNSUPPORTED, "1-hop pattern: more than 3839 two-hop candidates in a column"};
    int nt = cap <= 512 ? 128 : 256;
    size_t lds = (sizeof(uint64_t) + 2 * sizeof(double) + 3 * sizeof(int32_t)) * cap +
                 sizeof(int32_t) * (1 + nt + 1 + 256);
    auto kern = pattern_1hop_kernel<T>;
    DIAF_HIP_TRY(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds));
    hipLaunchKernelGGL(kern, dim3(ncols), dim3(nt), lds, st, n, Acp, Ari, Aval, ptop, cap, cols, cnt,
                       Jtmp);
    DIAF_HIP_TRY(hipGetLastError());
    return {};
}

template Err launch_pattern_1hop<double>(int, const int32_t*, const int32_t*, const double*, int,
                                         int, const int32_t*, int, int32_t*, int32_t*,
                                         hipStream_t);
template Err launch_pattern_1hop<zc>(int, const int32_t*, const int32_t*, const zc*, int, int,
                                     const int32_t*, int, int32_t*, int32_t*, hipStream_t);

}  // namespace diaf
