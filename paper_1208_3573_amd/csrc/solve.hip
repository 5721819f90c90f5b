// Apply M = W V^{-1} (eq. 2.1) and right-preconditioned BiCGSTAB
// (Section 5).
//
// * SpMV: CSR, one thread per row.
// * Triangular solve with V: sync-free, one wave per chunk of 256 rows.  A
//   chunk is taken from an atomic ticket in dependency order (ascending
//   rows for lower V, descending for upper V), so every row a wave waits on
//   belongs to the same wave or to a wave that started earlier.  Values
//   inside the chunk pass through LDS; values from earlier waves are read
//   from x itself, which is filled with a signalling-NaN sentinel before the
//   launch (a value is ready once it differs from the sentinel).  Waiting is
//   a wave-uniform polling loop with an iteration cap that raises an error
//   flag, so every wave always exits.
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

template <class T>
Err launch_spmv_csr(int n, const int32_t* rp, const int32_t* ci, const T* val, const T* x, T* y,
                    const int32_t* done, hipStream_t st)
{
    if (n == 0) return {};
    // lanes per row from the mean row length (read once per matrix on the host
    // would need a sync; the caller's matrices here are A (~7/row) and W)
    int64_t threads4 = (int64_t)n * 4;
    hipLaunchKernelGGL((spmv_csr_kernel<T, 4>), dim3((unsigned)((threads4 + 255) / 256)), dim3(256),
                       0, st, n, rp, ci, val, x, y, done);
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

template <class T>
__device__ inline bool load_ready(const T* x, int c, T& out)
{
    const uint64_t* p = (const uint64_t*)(x + c);
    if constexpr (num<T>::is_complex) {
        uint64_t a = ld_agent(p), b = ld_agent(p + 1);
        if (a == TRSV_SENTINEL || b == TRSV_SENTINEL) return false;
        out = T{__longlong_as_double((long long)a), __longlong_as_double((long long)b)};
    } else {
        uint64_t a = ld_agent(p);
        if (a == TRSV_SENTINEL) return false;
        out = __longlong_as_double((long long)a);
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

static constexpr int TRSV_SPIN_CAP = 1 << 22;

// Orders the LDS accesses of the lanes of one wave (LDS executes one wave's
// instructions in order, so this only has to stop the compiler from moving
// or caching accesses across it); unlike a workgroup barrier it does not
// wait for outstanding global stores.  LDS is accessed with plain loads and
// stores: a volatile access through a generic pointer becomes a flat access
// that waits on all outstanding memory operations.
__device__ inline void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    __asm__ __volatile__("" ::: "memory");
}

// A workgroup of NW waves owns NW x RPL x 64 consecutive rows (in dependency
// order); wave w the w-th block of RPL x 64 rows, lane l of it the rows l,
// l + 64, ... which it finishes one after the other.  Rows of the same chunk
// hand their values over through LDS whichever wave owns them.  At start
// the wave copies the right-hand side, the diagonal and the first
// trsv_dmax<T> off-diagonal entries of each of its rows into LDS (a longer
// row reads the rest from global memory when it gets there).  It then
// alternates (a) rounds that advance every row whose next dependency lies
// in the wave, through LDS, until none advances, and (b) one polling round
// on global memory for the rows blocked on another wave, so global latency
// is paid per hop between waves rather than per dependency step.  Entries
// are consumed in CSR order, so the result does not depend on timing.
template <class T>
struct trsv_dmax { static constexpr int v = num<T>::is_complex ? 6 : 8; };

template <class T, int NW, int RPL>
__global__ void __launch_bounds__(64 * NW) trsv_kernel(int n, const int32_t* rp, const int32_t* ci,
                                                  const T* val, int upper, const T* b, T* x,
                                                  TrsvCtl* ctl, const int32_t* done,
                                                  int sleep_cycles)
{
    if (done && *done) return;
    constexpr int WROWS = 64 * RPL;     // rows of one wave
    constexpr int ROWS = NW * WROWS;    // rows of the workgroup's chunk
    constexpr int DM = trsv_dmax<T>::v;
    __shared__ uint32_t s_chunk;
    __shared__ T sx[ROWS];         // right-hand side, then the solution
    __shared__ int sready[ROWS];
    __shared__ T sdg[ROWS];        // diagonal entry of each row
    __shared__ int snd[ROWS];      // off-diagonal entries held in LDS
    __shared__ int sov[ROWS];      // first entry not held in LDS (= row end if none)
    __shared__ int spe[ROWS];      // row end
    __shared__ int sdc[NW * RPL * DM * 64];
    __shared__ T sdv[NW * RPL * DM * 64];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    if (tid == 0) s_chunk = atomicAdd(&ctl->ticket, 1u);
    for (int k = tid; k < ROWS; k += 64 * NW) sready[k] = 0;
    __syncthreads();
    const int base = (int)s_chunk * ROWS;
    const int wbase = base + wv * WROWS;  // first row of this wave
    const int lbase = wv * WROWS;         // its slot in the chunk arrays
    const int dbase = wv * RPL;           // its rows in the entry lists
    const auto wrong_tri = [&](int c, int r) { return upper ? (c < r) : (c > r); };

    for (int qq = 0; qq < RPL; ++qq) {
        const int ps = wbase + qq * 64 + lane;
        if (ps >= n) break;
        const int ii = upper ? n - 1 - ps : ps;
        const int pe = rp[ii + 1];
        T dg = num<T>::one();
        int nd = 0, ov = pe;
        for (int pp = rp[ii]; pp < pe; ++pp) {
            const int c = ci[pp];
            if (c == ii) { dg = val[pp]; continue; }
            if (wrong_tri(c, ii)) continue;  // entries outside the triangle are ignored
            if (nd < DM) {
                sdc[((dbase + qq) * DM + nd) * 64 + lane] = c;
                sdv[((dbase + qq) * DM + nd) * 64 + lane] = val[pp];
                ++nd;
            } else if (ov == pe) {
                ov = pp;
            }
        }
        sx[lbase + qq * 64 + lane] = b[ii];
        sdg[lbase + qq * 64 + lane] = dg;
        snd[lbase + qq * 64 + lane] = nd;
        sov[lbase + qq * 64 + lane] = ov;
        spe[lbase + qq * 64 + lane] = pe;
    }
    __syncthreads();

    int q = 0;
    int pos = wbase + lane;
    bool fin = pos >= n;
    int i = 0, d = 0, nd = 0, ov = 0, pe = 0;
    T acc = num<T>::zero();
    const auto start_row = [&]() {
        const int k = lbase + q * 64 + lane;
        i = upper ? n - 1 - pos : pos;
        acc = sx[k];
        d = 0;
        nd = snd[k];
        ov = sov[k];
        pe = spe[k];
    };
    // next unconsumed dependency of the current row; false once none is left.
    // Consumption reads LDS only: when a long row has used up its LDS list,
    // the next entries are first copied there from global memory (so no
    // wait for global loads sits on the common path).
    const auto next_dep = [&](int& c, T& v) -> bool {
        if (d == nd) {
            if (ov >= pe) return false;
            int cnt = 0;
            for (; ov < pe && cnt < DM; ++ov) {
                const int cc = ci[ov];
                if (cc == i || wrong_tri(cc, i)) continue;
                sdc[((dbase + q) * DM + cnt) * 64 + lane] = cc;
                sdv[((dbase + q) * DM + cnt) * 64 + lane] = val[ov];
                ++cnt;
            }
            d = 0;
            nd = cnt;
            if (cnt == 0) return false;
        }
        c = sdc[((dbase + q) * DM + d) * 64 + lane];
        v = sdv[((dbase + q) * DM + d) * 64 + lane];
        return true;
    };
    const auto consume = [&]() { ++d; };
    if (!fin) start_row();

    int spins = 0;
    bool err = false;
    while (!__all(fin)) {
        // (a) LDS rounds
        for (;;) {
            bool prog = false;
            int done_slot = -1;
            if (!fin) {
                int c;
                T v;
                bool more;
                while ((more = next_dep(c, v))) {
                    const int cpos = upper ? n - 1 - c : c;
                    if (cpos < base) break;  // another chunk: polled in (b)
                    if (!__hip_atomic_load(&sready[cpos - base], __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_WORKGROUP))
                        break;
                    // the row may belong to another wave of the workgroup: its
                    // value is read only after its flag
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
                    acc -= v * sx[cpos - base];
                    consume();
                }
                if (!more) {
                    const int k = lbase + q * 64 + lane;
                    const T xi = div_t(acc, sdg[k]);
                    sx[k] = xi;
                    store_ready(x, i, xi);
                    done_slot = k;
                    prog = true;
                    spins = 0;
                    ++q;
                    pos += 64;
                    if (q == RPL || pos >= n) fin = true;
                    else start_row();
                }
            }
            wave_sync();
            if (done_slot >= 0) {
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
                __hip_atomic_store(&sready[done_slot], 1, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
            }
            wave_sync();
            if (!__any(prog)) break;
        }
        if (__all(fin)) break;
        // (b) one polling round for rows waiting on another wave
        bool polled = false;
        if (!fin) {
            int c;
            T v;
            while (next_dep(c, v)) {
                const int cpos = upper ? n - 1 - c : c;
                if (cpos >= base) break;  // inside the chunk: back to (a)
                T xc;
                if (!load_ready(x, c, xc)) break;
                acc -= v * xc;
                consume();
                polled = true;
            }
            if (!polled && ++spins > TRSV_SPIN_CAP) {
                err = true;
                fin = true;
            }
        }
        if (!__any(polled) && sleep_cycles) __builtin_amdgcn_s_sleep(1);
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
                T* x, TrsvCtl* ctl, const int32_t* done, TrsvTune tune, hipStream_t st)
{
    if (n == 0) return {};
    int64_t nw = (int64_t)n * words<T>::W;
    hipLaunchKernelGGL(fill_sentinel_kernel<T>, dim3((unsigned)((nw + 255) / 256)), dim3(256), 0, st,
                       n, x, done);
    if (num<T>::is_complex && tune.waves > 8) tune.waves = 8;  // LDS holds 8 x 64 complex rows
    if (tune.waves > 1) tune.rows_per_lane = 1;
    const int rows = 64 * tune.rows_per_lane * tune.waves;
    const dim3 grid((n + rows - 1) / rows);
#define TRSV_CASE(NW, RPL)                                                                       \
    if (tune.waves == NW && tune.rows_per_lane == RPL) {                                          \
        hipLaunchKernelGGL((trsv_kernel<T, NW, RPL>), grid, dim3(64 * NW), 0, st, n, rp, ci, val, \
                           upper, b, x, ctl, done, tune.backoff);                                 \
        DIAF_HIP_TRY(hipGetLastError());                                                          \
        return {};                                                                                \
    }
    TRSV_CASE(1, 1)
    TRSV_CASE(1, 2)
    TRSV_CASE(1, 4)
    TRSV_CASE(4, 1)
    TRSV_CASE(8, 1)
    if constexpr (!num<T>::is_complex) {
        TRSV_CASE(16, 1)
    }
#undef TRSV_CASE
    return {DIAF_EINVAL, "triangular solve: unsupported waves x rows-per-lane combination"};
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
                       uint32_t* ready, TrsvCtl* ctl, int32_t* maxlevel_dev, hipStream_t st)
{
    (void)ready;
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

__host__ __device__ inline int red_blocks(int n)
{
    int b = (n + RNT * 4 - 1) / (RNT * 4);
    return b < 1 ? 1 : (b > RBMAX ? RBMAX : b);
}

// Block-reduce NV doubles per thread into partial[blockIdx * NV + v]; returns
// true in the block that finished last (its threads then see all partials).
template <int NV>
__device__ inline bool reduce_partials(double (&vals)[NV], double* partial, uint32_t* ticket)
{
    __shared__ double red[NV][RNT];
    __shared__ bool last;
    for (int v = 0; v < NV; ++v) red[v][threadIdx.x] = vals[v];
    __syncthreads();
    for (int o = RNT / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o)
            for (int v = 0; v < NV; ++v) red[v][threadIdx.x] += red[v][threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        for (int v = 0; v < NV; ++v) partial[blockIdx.x * NV + v] = red[v][0];
        __threadfence();
        uint32_t t = atomicAdd(ticket, 1u);
        last = (t == gridDim.x - 1);
    }
    __syncthreads();
    if (last) __threadfence();
    return last;
}

// Sum of the per-block partials by the whole (last) block: a strided load
// per thread and a tree in LDS, both in a fixed order.
template <int NV>
__device__ inline void sum_partials(const double* partial, int nb, double (&out)[NV])
{
    __shared__ double red2[NV][RNT];
    for (int v = 0; v < NV; ++v) {
        double a = 0.0;
        for (int b = threadIdx.x; b < nb; b += RNT)
            a += __hip_atomic_load(&partial[b * NV + v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        red2[v][threadIdx.x] = a;
    }
    __syncthreads();
    for (int o = RNT / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o)
            for (int v = 0; v < NV; ++v) red2[v][threadIdx.x] += red2[v][threadIdx.x + o];
        __syncthreads();
    }
    for (int v = 0; v < NV; ++v) out[v] = red2[v][0];
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

template <class T>
__global__ void __launch_bounds__(RNT) bicg_init_kernel(BicgVecs<T> V, double tol, int maxit)
{
    double acc[1] = {0.0};
    BICG_GRID_LOOP {
        T bi = V.b[i];
        V.x[i] = num<T>::zero();
        V.r[i] = bi;
        V.rh[i] = bi;
        V.p[i] = num<T>::zero();
        V.v[i] = num<T>::zero();
        acc[0] += num<T>::abs2(bi);
    }
    if (reduce_partials<1>(acc, V.partial, &V.st->red_ticket)) {
        double s[1];
        sum_partials<1>(V.partial, gridDim.x, s);
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
    }
}

// rho = <rh, r>; beta; iteration count and the maxit stop.
template <class T>
__global__ void __launch_bounds__(RNT) bicg_rho_kernel(BicgVecs<T> V)
{
    if (V.st->done) return;
    double acc[2] = {0.0, 0.0};
    BICG_GRID_LOOP {
        T d = num<T>::cmul(V.rh[i], V.r[i]);
        acc[0] += num<T>::re(d);
        acc[1] += num<T>::im(d);
    }
    if (reduce_partials<2>(acc, V.partial, &V.st->red_ticket)) {
        double s[2];
        sum_partials<2>(V.partial, gridDim.x, s);
        if (threadIdx.x != 0) return;
        BicgState<T>* S = V.st;
        S->red_ticket = 0;
        T rho = mk2<T>(s[0], s[1]);
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

// x = x + alpha ph + omega sh; r = s - omega t; full-step convergence test.
template <class T>
__global__ void __launch_bounds__(RNT) bicg_xr_kernel(BicgVecs<T> V)
{
    if (V.st->done) return;
    const T alpha = V.st->alpha, omega = V.st->omega;
    double acc[1] = {0.0};
    BICG_GRID_LOOP {
        V.x[i] = V.x[i] + alpha * V.ph[i] + omega * V.sh[i];
        T r = V.s[i] - omega * V.t[i];
        V.r[i] = r;
        acc[0] += num<T>::abs2(r);
    }
    if (reduce_partials<1>(acc, V.partial, &V.st->red_ticket)) {
        double s[1];
        sum_partials<1>(V.partial, gridDim.x, s);
        if (threadIdx.x != 0) return;
        BicgState<T>* S = V.st;
        S->red_ticket = 0;
        double nr = sqrt(s[0]);
        S->res = nr / S->bnorm;
        S->rho_prev = S->rho;
        if (nr <= S->tol * S->bnorm) { S->done = 1; S->flag = 0; }
    }
}

// After the loop (and bicg_half_fix), with t = A x: ||b - A x|| / ||b||
// into st->tt.
template <class T>
__global__ void __launch_bounds__(RNT) bicg_true_res_kernel(BicgVecs<T> V)
{
    double acc[1] = {0.0};
    BICG_GRID_LOOP {
        T d = V.b[i] - V.t[i];
        acc[0] += num<T>::abs2(d);
    }
    if (reduce_partials<1>(acc, V.partial, &V.st->red_ticket)) {
        double s[1];
        sum_partials<1>(V.partial, gridDim.x, s);
        if (threadIdx.x != 0) return;
        V.st->red_ticket = 0;
        V.st->tt = V.st->bnorm > 0 ? sqrt(s[0]) / V.st->bnorm : 0.0;
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
template <class T> Err bicg_rho(const BicgVecs<T>& V, hipStream_t st) { LAUNCH_STAGE(bicg_rho_kernel) }
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
    template Err launch_spmv_csr<T>(int, const int32_t*, const int32_t*, const T*, const T*, T*,  \
                                    const int32_t*, hipStream_t);                                 \
    template Err launch_trsv<T>(int, const int32_t*, const int32_t*, const T*, int, const T*, T*, \
                                TrsvCtl*, const int32_t*, TrsvTune, hipStream_t);                 \
    template Err launch_diag_solve<T>(int, const int32_t*, const int32_t*, const T*, const T*,    \
                                      T*, const int32_t*, hipStream_t);                           \
    template Err bicg_init<T>(const BicgVecs<T>&, double, int, hipStream_t);                      \
    template Err bicg_rho<T>(const BicgVecs<T>&, hipStream_t);                                    \
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
