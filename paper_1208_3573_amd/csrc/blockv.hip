// Block diagonal V (paper Section 5: V the block diagonal matrices of the
// splitting A = L + D + U, blocks of consecutive rows and columns).
//
// V^{-1} in M = W V^{-1} (eq. 2.1) is applied block by block: after the
// factorization each diagonal block of V is copied into LDS and factored
// P V_b = L U by Gaussian elimination with partial pivoting (the largest
// modulus in the pivot column, the lowest row on ties), one wave per block
// and one lane per row (blocks of at most 64 rows).  The factors are stored
// densely, column-major, so that every step of the block solve reads one
// coalesced column.  The solve is again one wave per block: the permuted
// right-hand side in registers, 2 b sequential steps that broadcast the
// finished entry with a cross-lane shuffle, the factor columns read from
// global memory ahead of the chain.  Blocks are independent, so
// unlike the triangular solve there is no cross-block dependency at all.
#include "dcommon.h"
#include "factor_kernels.h"

namespace diaf {

namespace {

constexpr int BLD = 64;  // LDS leading dimension (rows per block at most)

__device__ inline double bdiv(double a, double b) { return a / b; }
__device__ inline zc bdiv(zc a, zc b)
{
    const double d = b.x * b.x + b.y * b.y;
    return {(a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d};
}
__device__ inline double bshfl(double v, int src) { return __shfl(v, src); }
__device__ inline zc bshfl(zc v, int src) { return {__shfl(v.x, src), __shfl(v.y, src)}; }

}  // namespace

// Pattern of D for column j: the rows of A(:, j) inside j's block.
__global__ void block_vpattern_kernel(int n, const int32_t* Acp, const int32_t* Ari,
                                      const int32_t* vblk, int32_t* cnt, const int32_t* Vcp,
                                      int32_t* Vri)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const int lo = vblk[2 * j], hi = vblk[2 * j + 1];
    int c = 0;
    for (int p = Acp[j]; p < Acp[j + 1]; ++p) {
        const int i = Ari[p];
        if (i >= lo && i < hi) {
            if (Vri) Vri[Vcp[j] + c] = i;
            ++c;
        }
    }
    if (!Vri) cnt[j] = c;
}

Err launch_block_vpattern(int n, const int32_t* Acp, const int32_t* Ari, const int32_t* vblk,
                          int32_t* cnt, const int32_t* Vcp, int32_t* Vri, hipStream_t st)
{
    if (n == 0) return {};
    hipLaunchKernelGGL(block_vpattern_kernel, dim3((n + 255) / 256), dim3(256), 0, st, n, Acp, Ari,
                       vblk, cnt, Vcp, Vri);
    DIAF_HIP_TRY(hipGetLastError());
    return {};
}

// LU of block b (rows bstart[b] .. bstart[b+1]-1) of the CSC V, stored at
// LU + boff[b] (column-major, b x b), the row permutation at perm[bstart[b]
// ..] (entry i: the block row that ends in position i).  *bad counts
// singular blocks (a zero pivot); bit 30 of *bad is set when V has an entry
// outside its block.
template <class T>
__global__ __launch_bounds__(64) void block_lu_kernel(const int32_t* bstart, const int64_t* boff,
                                                      const int32_t* Vcp, const int32_t* Vri,
                                                      const T* Vval, T* LU, int32_t* perm,
                                                      int32_t* bad)
{
    __shared__ T M[BLD * BLD];
    __shared__ T prow[BLD];
    __shared__ int32_t pv[BLD];
    __shared__ int32_t cpl[BLD + 1];
    __shared__ int s_sing;
    const int b = blockIdx.x;
    const int lane = threadIdx.x;
    const int b0 = bstart[b], bs = bstart[b + 1] - b0;
    for (int c = 0; c < bs; ++c) M[lane + c * BLD] = num<T>::zero();
    for (int i = lane; i <= bs; i += 64) cpl[i] = Vcp[b0 + i];
    pv[lane] = lane;
    if (lane == 0) s_sing = 0;
    __syncthreads();
    // the block's entries are contiguous in the CSC arrays: each lane takes
    // every 64th and finds its column by bisection of the column starts, so
    // all loads are independent
    for (int p = cpl[0] + lane; p < cpl[bs]; p += 64) {
        int lo = 0, hi = bs - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (cpl[mid] <= p)
                lo = mid;
            else
                hi = mid - 1;
        }
        const int i = Vri[p] - b0;
        if (i >= 0 && i < bs)
            M[i + lo * BLD] = Vval[p];
        else
            atomicOr(bad, 1 << 30);
    }
    __syncthreads();
    for (int c = 0; c < bs; ++c) {
        // pivot: the largest modulus on or below the diagonal, lowest row on ties
        double mv = lane >= c && lane < bs ? num<T>::abs2(M[lane + c * BLD]) : -1.0;
        if (mv != mv) mv = INFINITY;  // a NaN entry is chosen, then reported below
        int mi = lane;
        for (int o = 32; o > 0; o >>= 1) {
            const double ov = __shfl_xor(mv, o);
            const int oi = __shfl_xor(mi, o);
            if (ov > mv || (ov == mv && oi < mi)) {
                mv = ov;
                mi = oi;
            }
        }
        // every lane holds the same (mv, mi): the order is total
        if (!(mv > 0.0) || !num<T>::finite(M[mi + c * BLD])) {
            if (lane == 0) s_sing = 1;
            break;
        }
        if (mi != c) {
            if (lane < bs) {
                const T a = M[c + lane * BLD];
                M[c + lane * BLD] = M[mi + lane * BLD];
                M[mi + lane * BLD] = a;
            }
            if (lane == 0) {
                const int t = pv[c];
                pv[c] = pv[mi];
                pv[mi] = t;
            }
        }
        __syncthreads();
        // the pivot row in an array of its own, so that the update loop's
        // loads do not wait on its stores
        if (lane < bs) prow[lane] = M[c + lane * BLD];
        __syncthreads();
        if (lane > c && lane < bs) {
            const T l = bdiv(M[lane + c * BLD], prow[c]);
            M[lane + c * BLD] = l;
            for (int q = c + 1; q < bs; ++q) M[lane + q * BLD] -= l * prow[q];
        }
        __syncthreads();
    }
    __syncthreads();
    if (s_sing && lane == 0) atomicAdd(bad, 1);
    T* out = LU + boff[b];
    for (int c = 0; c < bs; ++c)
        if (lane < bs) out[lane + (size_t)c * bs] = M[lane + c * BLD];
    if (lane < bs) perm[b0 + lane] = pv[lane];
}

template <class T>
Err launch_block_lu(int nblk, const int32_t* bstart, const int64_t* boff, const int32_t* Vcp,
                    const int32_t* Vri, const T* Vval, T* LU, int32_t* perm, int32_t* bad,
                    hipStream_t st)
{
    if (nblk == 0) return {};
    hipLaunchKernelGGL(block_lu_kernel<T>, dim3(nblk), dim3(64), 0, st, bstart, boff, Vcp, Vri,
                       Vval, LU, perm, bad);
    DIAF_HIP_TRY(hipGetLastError());
    return {};
}

// t = V^{-1} x block by block with the stored LU factors (no-op once *done).
// Lane i keeps entry i of the permuted right-hand side in a register; step c
// broadcasts the finished entry c and every lane below (forward) or above
// (backward) subtracts its multiple.  The factor entries a lane needs do not
// depend on the running values, so they are read straight from global
// memory, one coalesced column per step, SB columns at a time into registers
// and double-buffered: the loads of the next SB columns are in flight while
// the shuffle chain works through the current ones.
constexpr int SB = 8;

template <class T>
__global__ __launch_bounds__(64) void block_solve_kernel(const int32_t* bstart,
                                                         const int64_t* boff, const T* LU,
                                                         const int32_t* perm, const T* x, T* t,
                                                         const int32_t* done)
{
    if (done && *done) return;
    const int b = blockIdx.x;
    const int lane = threadIdx.x;
    const int b0 = bstart[b], bs = bstart[b + 1] - b0;
    const bool act = lane < bs;
    const T* F = LU + boff[b];
    T z = act ? x[b0 + perm[b0 + lane]] : num<T>::zero();
    T cur[SB], nxt[SB];
    // L z = P x (unit lower triangular): columns 0 .. bs-2, below the diagonal
    const auto load_l = [&](int c0, T (&buf)[SB]) {
#pragma unroll
        for (int u = 0; u < SB; ++u) {
            const int c = c0 + u;
            buf[u] = act && lane > c && c < bs - 1 ? F[lane + (size_t)c * bs] : num<T>::zero();
        }
    };
    load_l(0, cur);
    for (int c0 = 0; c0 < bs - 1; c0 += SB) {
        if (c0 + SB < bs - 1) load_l(c0 + SB, nxt);
#pragma unroll
        for (int u = 0; u < SB; ++u) {
            const int c = c0 + u;
            if (c < bs - 1) {
                const T zc = bshfl(z, c);
                if (lane > c) z -= cur[u] * zc;
            }
        }
#pragma unroll
        for (int u = 0; u < SB; ++u) cur[u] = nxt[u];
    }
    // U t = z: columns bs-1 down to 0, on and above the diagonal
    const auto load_u = [&](int c0, T (&buf)[SB]) {
#pragma unroll
        for (int u = 0; u < SB; ++u) {
            const int c = c0 - u;
            buf[u] = act && c >= 0 && lane <= c ? F[lane + (size_t)c * bs] : num<T>::zero();
        }
    };
    load_u(bs - 1, cur);
    for (int c0 = bs - 1; c0 >= 0; c0 -= SB) {
        if (c0 - SB >= 0) load_u(c0 - SB, nxt);
#pragma unroll
        for (int u = 0; u < SB; ++u) {
            const int c = c0 - u;
            if (c >= 0) {
                if (lane == c) z = bdiv(z, cur[u]);
                const T tc = bshfl(z, c);
                if (lane < c) z -= cur[u] * tc;
            }
        }
#pragma unroll
        for (int u = 0; u < SB; ++u) cur[u] = nxt[u];
    }
    if (act) t[b0 + lane] = z;
}

template <class T>
Err launch_block_solve(int nblk, const int32_t* bstart, const int64_t* boff, const T* LU,
                       const int32_t* perm, const T* x, T* t, const int32_t* done, hipStream_t st)
{
    if (nblk == 0) return {};
    hipLaunchKernelGGL(block_solve_kernel<T>, dim3(nblk), dim3(64), 0, st, bstart, boff, LU, perm,
                       x, t, done);
    DIAF_HIP_TRY(hipGetLastError());
    return {};
}

template Err launch_block_lu<double>(int, const int32_t*, const int64_t*, const int32_t*,
                                     const int32_t*, const double*, double*, int32_t*, int32_t*,
                                     hipStream_t);
template Err launch_block_lu<zc>(int, const int32_t*, const int64_t*, const int32_t*,
                                 const int32_t*, const zc*, zc*, int32_t*, int32_t*, hipStream_t);
template Err launch_block_solve<double>(int, const int32_t*, const int64_t*, const double*,
                                        const int32_t*, const double*, double*, const int32_t*,
                                        hipStream_t);
template Err launch_block_solve<zc>(int, const int32_t*, const int64_t*, const zc*, const int32_t*,
                                    const zc*, zc*, const int32_t*, hipStream_t);

}  // namespace diaf
