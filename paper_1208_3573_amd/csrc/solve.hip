// Apply M = W V^{-1} (eq. 2.1) and right-preconditioned BiCGSTAB
// (Section 5).
//
// * SpMV: CSR, one thread per row.
// * Triangular solve with V: sync-free, one workgroup per chunk of 64 x NW
//   rows, one row per lane.  A chunk is taken from an atomic ticket in
//   dependency order (ascending rows for lower V, descending for upper V),
//   so every row a workgroup waits on belongs to its own chunk or to a chunk
//   taken earlier.  Values inside the chunk pass through LDS; values from
//   earlier chunks are read from x itself.  Both are filled with a
//   signalling-NaN sentinel first (a value is ready once it differs from the
//   sentinel).  Waiting is a wave-uniform polling loop with an iteration cap
//   that raises an error flag, so every wave always exits.
// * BiCGSTAB runs on the device: each stage is a kernel that returns at
//   once when the solve has finished, reductions are two-stage in a fixed
//   order (the last block to finish sums the per-block partials and updates
//   the scalar state), and the host only polls the state between batches of
//   iterations.
#include "dcommon.h"
#include "factor_kernels.h"

namespace diaf {

// ---------------------------------------------------------------------------
// SpMV y = X x (CSR)
// ---------------------------------------------------------------------------
template <class T, int G>
__global__ void __launch_bounds__(256) spmv_csr_kernel(int n, const int32_t* rp, const int32_t* ci,
                                                     const T* val, const T* x, T* y,
                                                     const int32_t* done)
{
    if (done && *done) return;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = t / G, g = t % G;
    T acc = num<T>::zero();
    if (i < n)
        for (int p = rp[i] + g; p < rp[i + 1]; p += G) acc += val[p] * x[ci[p]];
    // fixed-order combine of the G partial sums (lanes of one row are adjacent)
    for (int o = G / 2; o > 0; o >>= 1) {
        if constexpr (num<T>::is_complex) {
            acc.x += __shfl_xor(acc.x, o);
            acc.y += __shfl_xor(acc.y, o);
        } else {
            acc += __shfl_xor(acc, o);
        }
    }
    if (i < n && g == 0) y[i] = acc;
}

// Lanes per row: the smallest power of two, between 4 and 32, at which each
// lane takes about two entries of an average row (7 per row for the 3D
// stencil A: 4 lanes; about 25 for pattern(A^2): 16).  On the 64^3 problem
// this beat one entry per lane (8 and 32 lanes) by 0.8 ms per solve and
// four lanes for both by 1.1 ms.  The lanes of a row and their combining
// order depend only on the matrix.
template <class T>
Err launch_spmv_csr(int n, int64_t nnz, const int32_t* rp, const int32_t* ci, const T* val,
                    const T* x, T* y, const int32_t* done, hipStream_t st)
{
    if (n == 0) return {};
    const int64_t mean = (nnz + n - 1) / n;
    int g = 4;
    while (g < 32 && 2 * g < mean) g *= 2;
    const int64_t threads = (int64_t)n * g;
    const dim3 grid((unsigned)((threads + 255) / 256));
#define SPMV_CASE(G)                                                                       \
    if (g == G) {                                                                          \
        hipLaunchKernelGGL((spmv_csr_kernel<T, G>), grid, dim3(256), 0, st, n, rp, ci, val, \
                           x, y, done);                                                    \
    }
    SPMV_CASE(4)
    SPMV_CASE(8)
    SPMV_CASE(16)
    SPMV_CASE(32)
#undef SPMV_CASE
    DIAF_HIP_TRY(hipGetLastError());
    return {};
}

// ---------------------------------------------------------------------------
// Diagonal V
// ---------------------------------------------------------------------------
template <class T>
__global__ void diag_solve_kernel(int n, const int32_t* rp, const int32_t* ci, const T* val,
                                  const T* b, T* x, const int32_t* done)
{
    if (done && *done) return;
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    T d = num<T>::zero();
    for (int p = rp[i]; p < rp[i + 1]; ++p)
        if (ci[p] == i) d = val[p];
    T bi = b[i];
    if constexpr (num<T>::is_complex) {
        double den = d.x * d.x + d.y * d.y;
        x[i] = T{(bi.x * d.x + bi.y * d.y) / den, (bi.y * d.x - bi.x * d.y) / den};
    } else {
        x[i] = bi / d;
    }
}

template <class T>
Err launch_diag_solve(int n, const int32_t* rp, const int32_t* ci, const T* val, const T* b, T* x,
                      const int32_t* done, hipStream_t st)
{
    if (n == 0) return {};
    hipLaunchKernelGGL(diag_solve_kernel<T>, dim3((n + 255) / 256), dim3(256), 0, st, n, rp, ci,
                       val, b, x, done);
    DIAF_HIP_TRY(hipGetLastError());
    return {};
}

// ---------------------------------------------------------------------------
// Sync-free triangular solve
//
// The solution vector doubles as the readiness flag: before the solve it is
// filled with a NaN whose payload no arithmetic produces (the sentinel);
// a row is ready once its entry differs from the sentinel.  Entries are
// written and polled with relaxed agent-scope atomics (coherent across the
// chip's L2 slices without cache-wide fences), so the value and its
// readiness are one 64-bit access.  Rows waited on inside the same wave are
// read from LDS.
// ---------------------------------------------------------------------------
static constexpr uint64_t TRSV_SENTINEL = 0x7ff4d1af5e000001ull;

__device__ inline uint64_t ld_agent(const uint64_t* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void st_agent(uint64_t* p, uint64_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <class T>
struct words;
template <>
struct words<double> {
    static constexpr int W = 1;
};
template <>
struct words<zc> {
    static constexpr int W = 2;
};

template <class T>
__global__ void fill_sentinel_kernel(int n, T* x, const int32_t* done)
{
    if (done && *done) return;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    constexpr int W = words<T>::W;
    if (i < (int64_t)n * W) ((uint64_t*)x)[i] = TRSV_SENTINEL;
}

// Entry i of x = the not-ready sentinel (every word of it).
template <class T>
__device__ inline void set_sentinel(T* x, int i)
{
    constexpr int W = words<T>::W;
#pragma unroll
    for (int k = 0; k < W; ++k) ((uint64_t*)x)[(int64_t)i * W + k] = TRSV_SENTINEL;
}

// Polling of entry c of x in two steps: issue the load of its raw words now
// and examine them later, so that other work can run while it is in flight.
template <class T>
__device__ inline void poll_issue(const T* x, int c, uint64_t (&w)[words<T>::W])
{
    const uint64_t* p = (const uint64_t*)(x + c);
#pragma unroll
    for (int k = 0; k < words<T>::W; ++k) w[k] = ld_agent(p + k);
}

template <class T>
__device__ inline bool poll_value(const uint64_t (&w)[words<T>::W], T& out)
{
    if constexpr (num<T>::is_complex) {
        if (w[0] == TRSV_SENTINEL || w[1] == TRSV_SENTINEL) return false;
        out = T{__longlong_as_double((long long)w[0]), __longlong_as_double((long long)w[1])};
    } else {
        if (w[0] == TRSV_SENTINEL) return false;
        out = __longlong_as_double((long long)w[0]);
    }
    return true;
}

template <class T>
__device__ inline void store_ready(T* x, int i, T v)
{
    uint64_t* p = (uint64_t*)(x + i);
    if constexpr (num<T>::is_complex) {
        st_agent(p, (uint64_t)__double_as_longlong(v.x));
        st_agent(p + 1, (uint64_t)__double_as_longlong(v.y));
    } else {
        st_agent(p, (uint64_t)__double_as_longlong(v));
    }
}

template <class T>
__device__ inline T div_t(T a, T d)
{
    if constexpr (num<T>::is_complex) {
        double den = d.x * d.x + d.y * d.y;
        return T{(a.x * d.x + a.y * d.y) / den, (a.y * d.x - a.x * d.y) / den};
    } else {
        return a / d;
    }
}

// acc - a * b with the rounding spelled out (explicit fused multiply-adds),
// so that every call site rounds alike whatever the compiler contracts.
template <class T>
__device__ __forceinline__ T msub(T acc, T a, T b)
{
    if constexpr (num<T>::is_complex) {
        double re = __builtin_fma(-a.x, b.x, acc.x);
        re = __builtin_fma(a.y, b.y, re);
        double im = __builtin_fma(-a.x, b.y, acc.y);
        im = __builtin_fma(-a.y, b.x, im);
        return T{re, im};
    } else {
        return __builtin_fma(-a, b, acc);
    }
}

// 1 / d, and a * b with the rounding spelled out.
template <class T>
__device__ inline T recip_t(T d)
{
    if constexpr (num<T>::is_complex) {
        const double den = d.x * d.x + d.y * d.y;
        return T{d.x / den, -d.y / den};
    } else {
        return 1.0 / d;
    }
}

template <class T>
__device__ __forceinline__ T mul_t(T a, T b)
{
    if constexpr (num<T>::is_complex) {
        return T{__builtin_fma(a.x, b.x, -(a.y * b.y)), __builtin_fma(a.x, b.y, a.y * b.x)};
    } else {
        return a * b;
    }
}

static constexpr int TRSV_SPIN_CAP = 1 << 22;

// LDS copy of one solution entry, read and written as relaxed workgroup-scope
// atomics of 64-bit words: the sentinel doubles as the not-ready mark, so a
// value and its readiness are one access (a torn complex read shows a
// sentinel half and is taken as not ready).
template <class T>
__device__ inline bool lds_take(const T* sx, int k, T& out)
{
    const uint64_t* p = (const uint64_t*)(sx + k);
    uint64_t w[words<T>::W];
#pragma unroll
    for (int q = 0; q < words<T>::W; ++q)
        w[q] = __hip_atomic_load(p + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    return poll_value(w, out);
}

template <class T>
__device__ inline void lds_put(T* sx, int k, T v)
{
    uint64_t* p = (uint64_t*)(sx + k);
    if constexpr (num<T>::is_complex) {
        __hip_atomic_store(p, (uint64_t)__double_as_longlong(v.x), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_WORKGROUP);
        __hip_atomic_store(p + 1, (uint64_t)__double_as_longlong(v.y), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_WORKGROUP);
    } else {
        __hip_atomic_store(p, (uint64_t)__double_as_longlong(v), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_WORKGROUP);
    }
}

// Off-diagonal entries of a row held in LDS (more are copied in from
// global memory when these are used up).
template <class T>
struct trsv_dmax { static constexpr int v = num<T>::is_complex ? 6 : 8; };

// A workgroup of NW waves owns a chunk of NW x 64 consecutive rows in
// dependency order (ascending rows for lower V, descending for upper V);
// lane l of wave w owns row w * 64 + l of it.  The chunk is taken from an
// atomic ticket, so every row it waits on lies in the chunk or in a chunk
// taken earlier by a running workgroup.  The rows' dependencies are consumed
// in ascending dependency order, the same for every launch shape, so the
// result does not depend on the shape or on timing.
//
// Set-up: the chunk's solution slots in LDS are filled with the sentinel;
// each lane keeps its row's right-hand side, diagonal and running sum in
// registers and copies the first trsv_dmax<T> off-diagonal entries into LDS,
// each coded as a chunk-local index or, for a dependency in an earlier
// chunk, as ~column.  Then it repeats:
//  (b1) issue loads of the next one or two dependencies that lie in earlier
//       chunks (global x, also sentinel-filled);
//  (a)  rounds in which every lane consumes the chunk-local dependencies
//       whose values have appeared in LDS (one LDS read per waiting lane)
//       and finishes its row when none is left (x = sum times the
//       reciprocal of the diagonal), until a round makes no progress;
//  (b2) consume the polled values that were ready.
// The latency of a poll thus overlaps the LDS rounds.  Waiting is capped:
// a lane that waits TRSV_SPIN_CAP polling rounds sets the error flag, so
// every wave exits.
template <class T, int NW>
__global__ void __launch_bounds__(64 * NW) trsv_kernel(int n, const int32_t* rp, const int32_t* ci,
                                                  const T* val, int upper, const T* b, T* x,
                                                  TrsvCtl* ctl, const int32_t* done,
                                                  int sleep_cap)
{
    if (done && *done) return;
    constexpr int ROWS = NW * 64;
    // up to 8 waves the LDS holds twice as many entries per row, at 16 waves
    // half as many again for real values
    constexpr int DM = NW <= 8 ? 2 * trsv_dmax<T>::v
                               : (num<T>::is_complex ? trsv_dmax<T>::v : 3 * trsv_dmax<T>::v / 2);
    __shared__ uint32_t s_chunk;
    __shared__ T sx[ROWS];            // solution of the chunk's rows (sentinel until known)
    __shared__ int sl[NW * DM * 64];  // entry code: chunk-local index, or ~column
    __shared__ T sv[NW * DM * 64];    // entry value
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    if (tid == 0) s_chunk = atomicAdd(&ctl->ticket, 1u);
    for (int k = tid; k < ROWS; k += 64 * NW) {
        uint64_t* p = (uint64_t*)(sx + k);
#pragma unroll
        for (int q = 0; q < words<T>::W; ++q) p[q] = TRSV_SENTINEL;
    }
    __syncthreads();
    const int base = (int)s_chunk * ROWS;
    const int me = wv * 64 + lane;  // chunk-local index of this lane's row
    const int pos = base + me;
    bool fin = pos >= n;
    const int slot0 = wv * DM * 64 + lane;  // LDS entry e of this lane at slot0 + e * 64
    const int step = upper ? -1 : 1;        // CSR order that visits dependencies ascending
    int i = 0, d = 0, nd = 0, ov = 0, oend = 0;
    T acc = num<T>::zero(), dg = num<T>::one();  // dg: the diagonal, then its reciprocal
    // copies up to DM entries from CSR position ov on into the lane's LDS slots
    const auto refill = [&]() {
        int cnt = 0;
        for (; ov != oend && cnt < DM; ov += step) {
            const int c = ci[ov];
            if (c == i || (upper ? (c < i) : (c > i))) continue;  // outside the triangle
            const int cpos = upper ? n - 1 - c : c;
            sl[slot0 + cnt * 64] = cpos >= base ? cpos - base : ~c;
            sv[slot0 + cnt * 64] = val[ov];
            ++cnt;
        }
        d = 0;
        nd = cnt;
    };
    if (!fin) {
        i = upper ? n - 1 - pos : pos;
        acc = b[i];
        const int pb = rp[i], pe = rp[i + 1];
        for (int pp = pb; pp < pe; ++pp) {  // branch-free, so the loads overlap
            const T vv = val[pp];
            dg = ci[pp] == i ? vv : dg;
        }
        ov = upper ? pe - 1 : pb;
        oend = upper ? pb - 1 : pe;
        refill();
    }
    dg = recip_t(dg);
    int cur = 0;
    T cv = num<T>::zero();
    // entry d into (cur, cv); past the end it reads the last slot, which is
    // then never used (every use checks d < nd)
    const auto load_cur = [&]() {
        const int dd = d < DM ? d : DM - 1;
        cur = sl[slot0 + dd * 64];
        cv = sv[slot0 + dd * 64];
    };
    // after a consumed dependency: the next one, refilling from CSR if needed
    const auto advance = [&]() {
        ++d;
        if (__builtin_expect(d == nd && ov != oend, 0)) refill();
        load_cur();
    };
    load_cur();
    // all set-up loads complete here (vmcnt(0); expcnt and lgkmcnt not
    // waited on), so no wait for them is left inside the polling loop, where
    // it would also wait for the polls in flight
    __builtin_amdgcn_s_waitcnt(0xF70);
    __syncthreads();

    int spins = 0, nsleep = 0;
    bool err = false;
    while (!__all(fin)) {
        // (b1)
        int npend = 0;
        uint64_t pw0[words<T>::W], pw1[words<T>::W];
        T pv1 = num<T>::zero();
        if (!fin && d < nd && cur < 0) {
            poll_issue(x, ~cur, pw0);
            npend = 1;
            if (d + 1 < nd) {
                const int c1 = sl[slot0 + (d + 1) * 64];
                if (c1 < 0) {
                    poll_issue(x, ~c1, pw1);
                    pv1 = sv[slot0 + (d + 1) * 64];
                    npend = 2;
                }
            }
        }
        bool aprog = false;  // some round of (a) made progress
        // (a): each round tries two chunk-local dependencies per lane, as
        // straight-line code (every lane reads a valid LDS slot; lanes with
        // nothing to take read their own and ignore it), then finishes rows
        // with none left
        for (;;) {
            bool prog = false;
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                const bool want = !fin && npend == 0 && d < nd && cur >= 0;
                T xv;
                const bool ok = lds_take(sx, want ? cur : me, xv) && want;
                if (ok) {
                    acc = msub(acc, cv, xv);
                    advance();
                }
                prog = prog || ok;
            }
            if (!fin && npend == 0 && d >= nd) {
                const T xi = mul_t(acc, dg);
                lds_put(sx, me, xi);
                store_ready(x, i, xi);
                fin = true;
                prog = true;
            }
            if (!__any(prog)) break;
            aprog = true;
        }
        // (b2)
        bool polled = false;
        if (npend > 0) {
            T xc;
            if (poll_value(pw0, xc)) {
                acc = msub(acc, cv, xc);
                advance();
                polled = true;
                if (npend == 2 && poll_value(pw1, xc)) {
                    acc = msub(acc, pv1, xc);
                    advance();
                }
            }
        }
        if (!fin && !polled && ++spins > TRSV_SPIN_CAP) {
            err = true;
            fin = true;
        }
        // back-off: a wave that made no progress sleeps before polling again,
        // twice as long as the time before, up to sleep_cap units of 64
        // cycles (0: never), so that waves far from the dependency front
        // leave the issue slots to the ones at it
        if (aprog || __any(polled)) {
            nsleep = 0;
        } else if (sleep_cap > 0) {
            nsleep = nsleep == 0 ? 1 : min(2 * nsleep, sleep_cap);
            for (int z = 0; z < nsleep; ++z) __builtin_amdgcn_s_sleep(1);
        }
    }
    if (err) atomicOr(&ctl->error, 1u);
    __syncthreads();
    if (tid == 0) {
        uint32_t f = atomicAdd(&ctl->finished, 1u);
        if (f == gridDim.x - 1) {
            // last workgroup: reset the tickets for the next launch
            ctl->ticket = 0;
            ctl->finished = 0;
        }
    }
}

template <class T>
Err launch_trsv(int n, const int32_t* rp, const int32_t* ci, const T* val, int upper, const T* b,
                T* x, TrsvCtl* ctl, const int32_t* done, TrsvTune tune, hipStream_t st,
                bool prefilled)
{
    if (n == 0) return {};
    int64_t nw = (int64_t)n * words<T>::W;
    if (!prefilled)
        hipLaunchKernelGGL(fill_sentinel_kernel<T>, dim3((unsigned)((nw + 255) / 256)), dim3(256), 0,
                           st, n, x, done);
    const int rows = 64 * tune.waves;
    const dim3 grid((n + rows - 1) / rows);
#define TRSV_CASE(NW)                                                                         \
    if (tune.waves == NW) {                                                                   \
        hipLaunchKernelGGL((trsv_kernel<T, NW>), grid, dim3(64 * NW), 0, st, n, rp, ci, val, \
                           upper, b, x, ctl, done, tune.backoff);                             \
        DIAF_HIP_TRY(hipGetLastError());                                                      \
        return {};                                                                            \
    }
    TRSV_CASE(1)
    TRSV_CASE(2)
    TRSV_CASE(4)
    TRSV_CASE(8)
    TRSV_CASE(16)
#undef TRSV_CASE
    return {DIAF_EINVAL, "triangular solve: waves per workgroup must be 1, 2, 4, 8 or 16"};
}

template <class T>
Err launch_fill_sentinel(int n, T* x, hipStream_t st)
{
    if (n == 0) return {};
    int64_t nw = (int64_t)n * words<T>::W;
    hipLaunchKernelGGL(fill_sentinel_kernel<T>, dim3((unsigned)((nw + 255) / 256)), dim3(256), 0, st,
                       n, x, (const int32_t*)nullptr);
    DIAF_HIP_TRY(hipGetLastError());
    return {};
}

// Level of every row in the triangular dependency DAG (same sync-free
// scheme with -1 as the not-ready value and an integer max instead of the
// substitution); *maxlevel = depth.
__global__ void fill_minus1_kernel(int n, int32_t* a)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = -1;
}

__global__ void __launch_bounds__(64) trsv_levels_kernel(int n, const int32_t* rp,
                                                         const int32_t* ci, int upper,
                                                         int32_t* level, TrsvCtl* ctl,
                                                         int32_t* maxlevel)
{
    __shared__ uint32_t s_chunk;
    __shared__ int slv[64];
    const int lane = threadIdx.x;
    if (lane == 0) s_chunk = atomicAdd(&ctl->ticket, 1u);
    slv[lane] = -1;
    __syncthreads();
    const int base = (int)s_chunk * 64;
    const int pos = base + lane;
    bool fin = pos >= n;
    const int i = fin ? 0 : (upper ? n - 1 - pos : pos);
    int lv = 0;
    int p = fin ? 0 : rp[i];
    const int pe = fin ? 0 : rp[i + 1];
    int spins = 0;
    bool err = false;
    while (!__all(fin)) {
        if (!fin) {
            while (p < pe) {
                int c = ci[p];
                if (c == i || (upper ? (c < i) : (c > i))) { ++p; continue; }
                const int cpos = upper ? n - 1 - c : c;
                int lc = cpos >= base
                             ? slv[cpos - base]
                             : __hip_atomic_load(&level[c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (lc < 0) break;
                lv = max(lv, lc);
                ++p;
            }
            if (p == pe) {
                slv[lane] = lv + 1;
                __hip_atomic_store(&level[i], lv + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                atomicMax(maxlevel, lv + 1);
                fin = true;
            } else if (++spins > TRSV_SPIN_CAP) {
                err = true;
                fin = true;
            }
        }
        __syncthreads();
    }
    if (err) atomicOr(&ctl->error, 1u);
    __syncthreads();
    if (lane == 0) {
        uint32_t f = atomicAdd(&ctl->finished, 1u);
        if (f == gridDim.x - 1) {
            ctl->ticket = 0;
            ctl->finished = 0;
        }
    }
}

Err launch_trsv_levels(int n, const int32_t* rp, const int32_t* ci, int upper, int32_t* level,
                       TrsvCtl* ctl, int32_t* maxlevel_dev, hipStream_t st)
{
    if (n == 0) return {};
    hipLaunchKernelGGL(fill_minus1_kernel, dim3((n + 255) / 256), dim3(256), 0, st, n, level);
    hipLaunchKernelGGL(trsv_levels_kernel, dim3((n + 63) / 64), dim3(64), 0, st, n, rp, ci, upper,
                       level, ctl, maxlevel_dev);
    DIAF_HIP_TRY(hipGetLastError());
    return {};
}

// ---------------------------------------------------------------------------
// BiCGSTAB stages
// ---------------------------------------------------------------------------
static constexpr int RNT = 256;
static constexpr int RBMAX = 512;

// Blocks of a stage kernel: 8 entries per thread.  Every block passes the
// single reduction ticket (a serialised atomic), so fewer blocks shorten the
// tail; at 64^3 (n = 262144) 128 blocks beat 256 (4 per thread) and 64.
__host__ __device__ inline int red_blocks(int n)
{
    int b = (n + RNT * 8 - 1) / (RNT * 8);
    return b < 1 ? 1 : (b > RBMAX ? RBMAX : b);
}

// Sum over the block of NV doubles per thread, the same value in every
// thread: a butterfly of shuffles inside each wave (its lane 0 keeps the
// result), then the four wave sums in wave order.  Fixed order, one barrier.
template <int NV>
__device__ inline void block_sum(const double (&vals)[NV], double (&out)[NV])
{
    constexpr int NWV = RNT / 64;
    __shared__ double wsum[NV][NWV];
    for (int v = 0; v < NV; ++v) {
        double a = vals[v];
        for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o);
        if ((threadIdx.x & 63) == 0) wsum[v][threadIdx.x >> 6] = a;
    }
    __syncthreads();
    for (int v = 0; v < NV; ++v) {
        double a = wsum[v][0];
        for (int w = 1; w < NWV; ++w) a += wsum[v][w];
        out[v] = a;
    }
}

// Block-reduce NV doubles per thread into partial[blockIdx * NV + v]; returns
// true in the block that finished last (its threads then see all partials).
template <int NV>
__device__ inline bool reduce_partials(double (&vals)[NV], double* partial, uint32_t* ticket)
{
    __shared__ bool last;
    double tot[NV];
    block_sum<NV>(vals, tot);
    if (threadIdx.x == 0) {
        for (int v = 0; v < NV; ++v) partial[blockIdx.x * NV + v] = tot[v];
        __threadfence();
        uint32_t t = atomicAdd(ticket, 1u);
        last = (t == gridDim.x - 1);
    }
    __syncthreads();
    if (last) __threadfence();
    return last;
}

// Sum of the per-block partials by the whole (last) block: a strided load
// per thread, then block_sum, both in a fixed order.
template <int NV>
__device__ inline void sum_partials(const double* partial, int nb, double (&out)[NV])
{
    double a[NV];
    for (int v = 0; v < NV; ++v) {
        a[v] = 0.0;
        for (int b = threadIdx.x; b < nb; b += RNT)
            a[v] += __hip_atomic_load(&partial[b * NV + v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    block_sum<NV>(a, out);
}

template <class T>
__device__ inline T mk2(double re, double im)
{
    if constexpr (num<T>::is_complex) return T{re, im};
    else return re;
}

template <class T>
__device__ inline bool bad_scalar(T a)
{
    double m = num<T>::abs(a);
    return !(m > 1e-300) || !isfinite(m);
}

#define BICG_GRID_LOOP for (int i = blockIdx.x * RNT + threadIdx.x; i < V.n; i += gridDim.x * RNT)

// The start of an iteration, from rho = <rh, r> of its residual: the maxit
// stop, the iteration count, the breakdown test and beta (by the last block
// of the stage that computed rho).
template <class T>
__device__ inline void bicg_begin_iteration(BicgState<T>* S, T rho)
{
    if (S->it + 1 > S->maxit) { S->done = 1; S->flag = 1; return; }
    S->it += 1;
    if (bad_scalar(rho)) { S->done = 1; S->flag = 2; return; }
    S->rho = rho;
    if (S->it == 1) {
        S->beta = num<T>::zero();
    } else {
        T q = div_t(rho, S->rho_prev);
        T a = div_t(S->alpha, S->omega);
        S->beta = q * a;
    }
}

// x = 0, r = rh = b, ||b||, and the first iteration's rho = <rh, r>.
template <class T>
__global__ void __launch_bounds__(RNT) bicg_init_kernel(BicgVecs<T> V, double tol, int maxit)
{
    double acc[3] = {0.0, 0.0, 0.0};
    BICG_GRID_LOOP {
        T bi = V.b[i];
        V.x[i] = num<T>::zero();
        V.r[i] = bi;
        V.rh[i] = bi;
        V.p[i] = num<T>::zero();
        V.v[i] = num<T>::zero();
        acc[0] += num<T>::abs2(bi);
        T d = num<T>::cmul(bi, bi);
        acc[1] += num<T>::re(d);
        acc[2] += num<T>::im(d);
    }
    if (reduce_partials<3>(acc, V.partial, &V.st->red_ticket)) {
        double s[3];
        sum_partials<3>(V.partial, gridDim.x, s);
        if (threadIdx.x != 0) return;
        BicgState<T>* S = V.st;
        S->bnorm = sqrt(s[0]);
        S->tol = tol;
        S->maxit = maxit;
        S->it = 0;
        S->rho_prev = num<T>::one();
        S->alpha = num<T>::one();
        S->omega = num<T>::one();
        S->beta = num<T>::zero();
        S->half = 0;
        S->omega_bad = 0;
        S->res = 1.0;
        S->done = (s[0] == 0.0) ? 1 : 0;
        S->flag = (s[0] == 0.0) ? 0 : 1;
        S->red_ticket = 0;
        if (!S->done) bicg_begin_iteration(S, mk2<T>(s[1], s[2]));
    }
}

template <class T>
__global__ void __launch_bounds__(RNT) bicg_p_kernel(BicgVecs<T> V)
{
    if (V.st->done) return;
    const T beta = V.st->beta, omega = V.st->omega;
    const bool first = V.st->it == 1;
    BICG_GRID_LOOP {
        V.p[i] = first ? V.r[i] : V.r[i] + beta * (V.p[i] - omega * V.v[i]);
    }
}

template <class T>
__global__ void __launch_bounds__(RNT) bicg_alpha_kernel(BicgVecs<T> V)
{
    if (V.st->done) return;
    double acc[2] = {0.0, 0.0};
    BICG_GRID_LOOP {
        T d = num<T>::cmul(V.rh[i], V.v[i]);
        acc[0] += num<T>::re(d);
        acc[1] += num<T>::im(d);
        if (V.clr_a) set_sentinel(V.clr_a, i);
    }
    if (reduce_partials<2>(acc, V.partial, &V.st->red_ticket)) {
        double s[2];
        sum_partials<2>(V.partial, gridDim.x, s);
        if (threadIdx.x != 0) return;
        BicgState<T>* S = V.st;
        S->red_ticket = 0;
        T rv = mk2<T>(s[0], s[1]);
        if (bad_scalar(rv)) { S->done = 1; S->flag = 2; return; }
        S->alpha = div_t(S->rho, rv);
    }
}

// s = r - alpha v; half-step convergence test (the x update of a half step
// is applied by bicg_half_fix after the loop).
template <class T>
__global__ void __launch_bounds__(RNT) bicg_s_kernel(BicgVecs<T> V)
{
    if (V.st->done) return;
    const T alpha = V.st->alpha;
    double acc[1] = {0.0};
    BICG_GRID_LOOP {
        T s = V.r[i] - alpha * V.v[i];
        V.s[i] = s;
        acc[0] += num<T>::abs2(s);
    }
    if (reduce_partials<1>(acc, V.partial, &V.st->red_ticket)) {
        double s[1];
        sum_partials<1>(V.partial, gridDim.x, s);
        if (threadIdx.x != 0) return;
        BicgState<T>* S = V.st;
        S->red_ticket = 0;
        double nr = sqrt(s[0]);
        S->res = nr / S->bnorm;
        if (nr <= S->tol * S->bnorm) { S->done = 1; S->flag = 0; S->half = 1; }
    }
}

template <class T>
__global__ void __launch_bounds__(RNT) bicg_omega_kernel(BicgVecs<T> V)
{
    if (V.st->done) return;
    double acc[3] = {0.0, 0.0, 0.0};
    BICG_GRID_LOOP {
        T ti = V.t[i];
        T d = num<T>::cmul(ti, V.s[i]);
        acc[0] += num<T>::re(d);
        acc[1] += num<T>::im(d);
        acc[2] += num<T>::abs2(ti);
    }
    if (reduce_partials<3>(acc, V.partial, &V.st->red_ticket)) {
        double s[3];
        sum_partials<3>(V.partial, gridDim.x, s);
        if (threadIdx.x != 0) return;
        BicgState<T>* S = V.st;
        S->red_ticket = 0;
        T ts = mk2<T>(s[0], s[1]);
        T om = div_t(ts, mk2<T>(s[2], 0.0));
        S->omega = om;
        if (bad_scalar(om)) { S->done = 1; S->flag = 2; S->half = 2; }
    }
}

// x = x + alpha ph + omega sh; r = s - omega t; full-step convergence test;
// the next iteration's rho = <rh, r> in the same pass.
template <class T>
__global__ void __launch_bounds__(RNT) bicg_xr_kernel(BicgVecs<T> V)
{
    if (V.st->done) return;
    const T alpha = V.st->alpha, omega = V.st->omega;
    double acc[3] = {0.0, 0.0, 0.0};
    BICG_GRID_LOOP {
        V.x[i] = V.x[i] + alpha * V.ph[i] + omega * V.sh[i];
        T r = V.s[i] - omega * V.t[i];
        V.r[i] = r;
        acc[0] += num<T>::abs2(r);
        T d = num<T>::cmul(V.rh[i], r);
        acc[1] += num<T>::re(d);
        acc[2] += num<T>::im(d);
        if (V.clr_x) set_sentinel(V.clr_x, i);
    }
    if (reduce_partials<3>(acc, V.partial, &V.st->red_ticket)) {
        double s[3];
        sum_partials<3>(V.partial, gridDim.x, s);
        if (threadIdx.x != 0) return;
        BicgState<T>* S = V.st;
        S->red_ticket = 0;
        double nr = sqrt(s[0]);
        S->res = nr / S->bnorm;
        S->rho_prev = S->rho;
        if (nr <= S->tol * S->bnorm) { S->done = 1; S->flag = 0; return; }
        bicg_begin_iteration(S, mk2<T>(s[1], s[2]));
    }
}

// After the loop (and bicg_half_fix), with t = A x: ||b - A x|| / ||b||
// into st->tt (||b|| summed here: under left preconditioning st->bnorm is
// the norm of M b).
template <class T>
__global__ void __launch_bounds__(RNT) bicg_true_res_kernel(BicgVecs<T> V)
{
    double acc[2] = {0.0, 0.0};
    BICG_GRID_LOOP {
        const T bi = V.b[i];
        T d = bi - V.t[i];
        acc[0] += num<T>::abs2(d);
        acc[1] += num<T>::abs2(bi);
    }
    if (reduce_partials<2>(acc, V.partial, &V.st->red_ticket)) {
        double s[2];
        sum_partials<2>(V.partial, gridDim.x, s);
        if (threadIdx.x != 0) return;
        V.st->red_ticket = 0;
        V.st->tt = s[1] > 0 ? sqrt(s[0]) / sqrt(s[1]) : 0.0;
    }
}

template <class T>
__global__ void __launch_bounds__(RNT) bicg_half_fix_kernel(BicgVecs<T> V)
{
    // half == 1: converged at the half step, x = x + alpha ph.
    // half == 2: omega breakdown, x = x + alpha ph as well.
    if (V.st->half == 0) return;
    const T alpha = V.st->alpha;
    BICG_GRID_LOOP { V.x[i] = V.x[i] + alpha * V.ph[i]; }
}

#define LAUNCH_STAGE(kern, ...)                                                              \
    hipLaunchKernelGGL(kern<T>, dim3(red_blocks(V.n)), dim3(RNT), 0, st, V, ##__VA_ARGS__);  \
    DIAF_HIP_TRY(hipGetLastError());                                                         \
    return {};

template <class T> Err bicg_init(const BicgVecs<T>& V, double tol, int maxit, hipStream_t st) { LAUNCH_STAGE(bicg_init_kernel, tol, maxit) }
template <class T> Err bicg_update_p(const BicgVecs<T>& V, hipStream_t st) { LAUNCH_STAGE(bicg_p_kernel) }
template <class T> Err bicg_alpha(const BicgVecs<T>& V, hipStream_t st) { LAUNCH_STAGE(bicg_alpha_kernel) }
template <class T> Err bicg_s(const BicgVecs<T>& V, hipStream_t st) { LAUNCH_STAGE(bicg_s_kernel) }
template <class T> Err bicg_omega(const BicgVecs<T>& V, hipStream_t st) { LAUNCH_STAGE(bicg_omega_kernel) }
template <class T> Err bicg_xr(const BicgVecs<T>& V, hipStream_t st) { LAUNCH_STAGE(bicg_xr_kernel) }
template <class T>
Err bicg_true_residual(const BicgVecs<T>& V, hipStream_t st)
{
    // caller has put A x in V.t after bicg_half_fix
    LAUNCH_STAGE(bicg_true_res_kernel)
}
template <class T>
Err bicg_half_fix(const BicgVecs<T>& V, hipStream_t st) { LAUNCH_STAGE(bicg_half_fix_kernel) }

#define INST(T)                                                                                   \
    template Err launch_spmv_csr<T>(int, int64_t, const int32_t*, const int32_t*, const T*,        \
                                    const T*, T*, const int32_t*, hipStream_t);                   \
    template Err launch_trsv<T>(int, const int32_t*, const int32_t*, const T*, int, const T*, T*, \
                                TrsvCtl*, const int32_t*, TrsvTune, hipStream_t, bool);           \
    template Err launch_fill_sentinel<T>(int, T*, hipStream_t);                                   \
    template Err launch_diag_solve<T>(int, const int32_t*, const int32_t*, const T*, const T*,    \
                                      T*, const int32_t*, hipStream_t);                           \
    template Err bicg_init<T>(const BicgVecs<T>&, double, int, hipStream_t);                      \
    template Err bicg_update_p<T>(const BicgVecs<T>&, hipStream_t);                               \
    template Err bicg_alpha<T>(const BicgVecs<T>&, hipStream_t);                                  \
    template Err bicg_s<T>(const BicgVecs<T>&, hipStream_t);                                      \
    template Err bicg_omega<T>(const BicgVecs<T>&, hipStream_t);                                  \
    template Err bicg_xr<T>(const BicgVecs<T>&, hipStream_t);                                     \
    template Err bicg_true_residual<T>(const BicgVecs<T>&, hipStream_t);                          \
    template Err bicg_half_fix<T>(const BicgVecs<T>&, hipStream_t);
INST(double)
INST(zc)
#undef INST

}  // namespace diaf
