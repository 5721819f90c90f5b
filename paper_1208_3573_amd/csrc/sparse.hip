// Sparse utilities: scans, V assembly (padded columns -> CSC), CSC -> CSR
// transposes (stable radix sort by row), input validation and per-column statistics.
#include <hipcub/hipcub.hpp>

#include "dcommon.h"
#include "factor_kernels.h"

namespace diaf {

// ---------------------------------------------------------------------------
// Exclusive scan (out has n+1 entries, out[n] = total).
// ---------------------------------------------------------------------------
__global__ void shift_kernel(const int32_t* in, int32_t* tmp, int n)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) tmp[i] = in[i];
    if (i == n) tmp[i] = 0;
}

Err exclusive_scan_i32(const int32_t* in, int32_t* out, int n, hipStream_t st)
{
    // out[0..n] = exclusive prefix sums of in[0..n) followed by the total:
    // scan n+1 values with a trailing zero.
    int32_t* tmp = nullptr;
    DIAF_TRY(amalloc((void**)&tmp, sizeof(int32_t) * (n + 1), st));
    hipLaunchKernelGGL(shift_kernel, dim3((n + 1 + 255) / 256), dim3(256), 0, st, in, tmp, n);
    size_t bytes = 0;
    DIAF_HIP_TRY(hipcub::DeviceScan::ExclusiveSum(nullptr, bytes, tmp, out, n + 1, st));
    void* ws = nullptr;
    DIAF_TRY(amalloc(&ws, bytes, st));
    DIAF_HIP_TRY(hipcub::DeviceScan::ExclusiveSum(ws, bytes, tmp, out, n + 1, st));
    afree(ws, st);
    afree(tmp, st);
    return {};
}

// ---------------------------------------------------------------------------
// V assembly: padded (n x lmax, -1 padded, rows sorted) -> CSC.
// ---------------------------------------------------------------------------
template <class T>
__global__ void compact_v_kernel(int n, int lmax, const int32_t* lcount, const int32_t* Vcp,
                                 const int32_t* Vrows, const T* Vvals, int32_t* Vri, T* Vval)
{
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)n * lmax) return;
    int j = (int)(idx / lmax), t = (int)(idx % lmax);
    if (t < lcount[j]) {
        Vri[Vcp[j] + t] = Vrows[idx];
        Vval[Vcp[j] + t] = Vvals[idx];
    }
}

template <class T>
Err launch_compact_v(int n, int lmax, const int32_t* lcount, const int32_t* Vcp,
                     const int32_t* Vrows, const T* Vvals, int32_t* Vri, T* Vval, hipStream_t st)
{
    int64_t tot = (int64_t)n * lmax;
    if (tot == 0) return {};
    hipLaunchKernelGGL(compact_v_kernel<T>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st,
                       n, lmax, lcount, Vcp, Vrows, Vvals, Vri, Vval);
    DIAF_HIP_TRY(hipGetLastError());
    return {};
}

// ---------------------------------------------------------------------------
// CSC -> CSR: count entries per row, scan, scatter, then sort each row by
// column so the result does not depend on the scatter order.
// ---------------------------------------------------------------------------
__global__ void row_count_kernel(int64_t nnz, const int32_t* ri, int32_t* cnt)
{
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < nnz) atomicAdd(&cnt[ri[p]], 1);
}

__global__ void iota_kernel(int64_t nnz, int32_t* v)
{
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < nnz) v[p] = (int32_t)p;
}

// Entry q of the CSR result comes from CSC position perm[q]; its column is
// found by a binary search in the column pointers.
template <class T>
__global__ void gather_csr_kernel(int n, int64_t nnz, const int32_t* cp, const T* val,
                                  const int32_t* perm, int32_t* ci, T* cval)
{
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nnz) return;
    const int32_t p = perm[q];
    int lo = 0, hi = n - 1;  // last column j with cp[j] <= p
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (cp[mid] <= p) lo = mid;
        else hi = mid - 1;
    }
    ci[q] = lo;
    cval[q] = val[p];
}

// CSC -> CSR: row counts and their scan give the row pointers; a stable
// radix sort of the entries by row (CSC order already has the columns
// ascending within every row, and stability keeps them so) gives the order.
template <class T>
Err csc_to_csr(int n, int64_t nnz, const int32_t* cp, const int32_t* ri, const T* val,
               int32_t* rp, int32_t* ci, T* cval, hipStream_t st)
{
    int32_t* cnt = nullptr;
    DIAF_TRY(amalloc((void**)&cnt, sizeof(int32_t) * (n + 1), st));
    DIAF_HIP_TRY(hipMemsetAsync(cnt, 0, sizeof(int32_t) * (n + 1), st));
    if (nnz > 0)
        hipLaunchKernelGGL(row_count_kernel, dim3((unsigned)((nnz + 255) / 256)), dim3(256), 0, st,
                           nnz, ri, cnt);
    DIAF_TRY(exclusive_scan_i32(cnt, rp, n, st));
    afree(cnt, st);
    if (nnz == 0) return {};
    int32_t *kout = nullptr, *vin = nullptr, *vout = nullptr;
    DIAF_TRY(amalloc((void**)&kout, sizeof(int32_t) * nnz, st));
    DIAF_TRY(amalloc((void**)&vin, sizeof(int32_t) * nnz, st));
    DIAF_TRY(amalloc((void**)&vout, sizeof(int32_t) * nnz, st));
    const unsigned blocks = (unsigned)((nnz + 255) / 256);
    hipLaunchKernelGGL(iota_kernel, dim3(blocks), dim3(256), 0, st, nnz, vin);
    int bits = 1;
    while ((1ll << bits) < (int64_t)n) ++bits;
    size_t tmp_bytes = 0;
    DIAF_HIP_TRY(hipcub::DeviceRadixSort::SortPairs(nullptr, tmp_bytes, ri, kout, vin, vout,
                                                    (int)nnz, 0, bits, st));
    void* tmp = nullptr;
    DIAF_TRY(amalloc(&tmp, tmp_bytes, st));
    DIAF_HIP_TRY(hipcub::DeviceRadixSort::SortPairs(tmp, tmp_bytes, ri, kout, vin, vout, (int)nnz,
                                                    0, bits, st));
    hipLaunchKernelGGL(gather_csr_kernel<T>, dim3(blocks), dim3(256), 0, st, n, nnz, cp, val, vout,
                       ci, cval);
    DIAF_HIP_TRY(hipGetLastError());
    afree(tmp, st);
    afree(kout, st);
    afree(vin, st);
    afree(vout, st);
    return {};
}

// ---------------------------------------------------------------------------
// Validation.  Codes: 1 colptr not monotone / out of range, 2 row out of
// range, 3 rows unsorted or duplicated, 4 diagonal missing, 5 non-finite
// value.  The smallest code seen wins (atomicMin over codes, 0 = fine).
// ---------------------------------------------------------------------------
template <class T>
__global__ void validate_kernel(int n, const int32_t* cp, const int32_t* ri, const T* val,
                                int need_diag, int32_t* bad)
{
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    int b = cp[j], e = cp[j + 1];
    int code = 0;
    if (e < b || b < 0) code = 1;
    int has_diag = 0;
    if (!code) {
        for (int p = b; p < e; ++p) {
            int i = ri[p];
            if (i < 0 || i >= n) { code = 2; break; }
            if (p > b && ri[p - 1] >= i) { code = 3; break; }
            if (i == j) has_diag = 1;
            if (val && !num<T>::finite(val[p])) { code = 5; break; }
        }
    }
    if (!code && need_diag && !has_diag) code = 4;
    if (code) atomicMin(bad, code);
}

template <class T>
Err launch_validate_csc(int n, const int32_t* cp, const int32_t* ri, const T* val,
                        int32_t* bad_dev, hipStream_t st)
{
    hipLaunchKernelGGL(validate_kernel<T>, dim3((n + 255) / 256), dim3(256), 0, st, n, cp, ri, val,
                       1, bad_dev);
    DIAF_HIP_TRY(hipGetLastError());
    return {};
}

Err launch_validate_pattern(int n, const int32_t* cp, const int32_t* ri, int need_diag,
                            int32_t* bad_dev, hipStream_t st)
{
    hipLaunchKernelGGL(validate_kernel<double>, dim3((n + 255) / 256), dim3(256), 0, st, n, cp, ri,
                       (const double*)nullptr, need_diag, bad_dev);
    DIAF_HIP_TRY(hipGetLastError());
    return {};
}

// ---------------------------------------------------------------------------
// Flag counts (bits 0..6) and sum of r_j^2 (two-stage, fixed order).
// ---------------------------------------------------------------------------
__global__ void flag_stats_kernel(int n, const uint32_t* flags, const double* r, int32_t* counts,
                                  double* partial)
{
    __shared__ double red[256];
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    double s = 0.0;
    if (j < n) {
        uint32_t f = flags[j];
        for (int b = 0; b < 8; ++b)
            if (f & (1u << b)) atomicAdd(&counts[b], 1);
        s = r[j] * r[j];
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void sum_partials_kernel(int nb, const double* partial, double* out)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double s = 0.0;
        for (int b = 0; b < nb; ++b) s += partial[b];
        *out = s;
    }
}

template <class T>
Err launch_flag_stats(int n, const uint32_t* flags, const double* r, int32_t* counts_dev,
                      double* nrm2_dev, hipStream_t st)
{
    int nb = (n + 255) / 256;
    double* partial = nullptr;
    DIAF_TRY(amalloc((void**)&partial, sizeof(double) * (nb + 1), st));
    hipLaunchKernelGGL(flag_stats_kernel, dim3(nb), dim3(256), 0, st, n, flags, r, counts_dev,
                       partial);
    hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(64), 0, st, nb, partial, nrm2_dev);
    DIAF_HIP_TRY(hipGetLastError());
    afree(partial, st);
    return {};
}

// Diagonal dominance of each V column in the padded per-column layout:
// dom[j] = |v_jj| / sum_{i != j} |v_ij| (infinite without off-diagonal
// entries, 0 without a diagonal entry).
template <class T>
__global__ void col_dominance_kernel(int n, int lmax, const int32_t* Vrows, const T* Vvals,
                                     const int32_t* lcount, double* dom)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    double d = 0.0, off = 0.0;
    const int l = lcount[j];
    for (int t = 0; t < l; ++t) {
        const int r = Vrows[(size_t)j * lmax + t];
        const double a = num<T>::abs(Vvals[(size_t)j * lmax + t]);
        if (r == j) d = a;
        else off += a;
    }
    dom[j] = off > 0.0 ? d / off : (d > 0.0 ? INFINITY : 0.0);
}

template <class T>
Err launch_col_dominance(int n, int lmax, const int32_t* Vrows, const T* Vvals,
                         const int32_t* lcount, double* dom, hipStream_t st)
{
    if (n == 0) return {};
    hipLaunchKernelGGL(col_dominance_kernel<T>, dim3((n + 255) / 256), dim3(256), 0, st, n, lmax,
                       Vrows, Vvals, lcount, dom);
    DIAF_HIP_TRY(hipGetLastError());
    return {};
}

#define INST(T)                                                                                  \
    template Err launch_col_dominance<T>(int, int, const int32_t*, const T*, const int32_t*,     \
                                         double*, hipStream_t);                                  \
    template Err launch_compact_v<T>(int, int, const int32_t*, const int32_t*, const int32_t*,  \
                                     const T*, int32_t*, T*, hipStream_t);                       \
    template Err csc_to_csr<T>(int, int64_t, const int32_t*, const int32_t*, const T*, int32_t*, \
                               int32_t*, T*, hipStream_t);                                       \
    template Err launch_validate_csc<T>(int, const int32_t*, const int32_t*, const T*, int32_t*, \
                                        hipStream_t);                                            \
    template Err launch_flag_stats<T>(int, const uint32_t*, const double*, int32_t*, double*,    \
                                      hipStream_t);
INST(double)
INST(zc)
#undef INST

// ---------------------------------------------------------------------------
// Zero, missing or non-finite diagonal entries of a CSR matrix (pivots of
// the triangular solve with V).
// ---------------------------------------------------------------------------
template <class T>
__global__ void diag_check_kernel(int n, const int32_t* rp, const int32_t* ci, const T* val,
                                  int32_t* bad)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    bool ok = false;
    for (int p = rp[i]; p < rp[i + 1]; ++p)
        if (ci[p] == i) ok = !num<T>::iszero(val[p]) && num<T>::finite(val[p]);
    if (!ok) atomicAdd(bad, 1);
}

template <class T>
Err launch_diag_check(int n, const int32_t* rp, const int32_t* ci, const T* val, int32_t* bad_dev,
                      hipStream_t st)
{
    if (n == 0) return {};
    hipLaunchKernelGGL(diag_check_kernel<T>, dim3((n + 255) / 256), dim3(256), 0, st, n, rp, ci,
                       val, bad_dev);
    DIAF_HIP_TRY(hipGetLastError());
    return {};
}
template Err launch_diag_check<double>(int, const int32_t*, const int32_t*, const double*, int32_t*,
                                       hipStream_t);
template Err launch_diag_check<zc>(int, const int32_t*, const int32_t*, const zc*, int32_t*,
                                   hipStream_t);

// v <- conj(v) (nothing to do for real values).
__global__ void conj_kernel(int64_t n, zc* v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) v[i].y = -v[i].y;
}

template <class T>
Err launch_conj(int64_t n, T* v, hipStream_t st)
{
    if constexpr (num<T>::is_complex) {
        if (n == 0) return {};
        hipLaunchKernelGGL(conj_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, v);
        DIAF_HIP_TRY(hipGetLastError());
    }
    return {};
}
template Err launch_conj<double>(int64_t, double*, hipStream_t);
template Err launch_conj<zc>(int64_t, zc*, hipStream_t);


// Order-independent 64-bit hash of a CSC pattern: the sum over all entries
// of a mix of (position, value), colptr and rowidx hashed with different
// salts.  A fingerprint for detecting a changed pattern, not a checksum of
// any strength beyond that.
__device__ inline uint64_t mix64(uint64_t x)
{
    x ^= x >> 30;
    x *= 0xbf58476d1ce4e5b9ull;
    x ^= x >> 27;
    x *= 0x94d049bb133111ebull;
    x ^= x >> 31;
    return x;
}

__global__ void pattern_hash_kernel(int n, int64_t nnz, const int32_t* cp, const int32_t* ri,
                                    unsigned long long* out)
{
    uint64_t h = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i <= n + nnz;
         i += (int64_t)gridDim.x * blockDim.x) {
        if (i <= n)
            h += mix64(((uint64_t)i << 32) ^ (uint32_t)cp[i] ^ 0x5851f42d4c957f2dull);
        else
            h += mix64((((uint64_t)(i - n - 1)) << 32) ^ (uint32_t)ri[i - n - 1]);
    }
    for (int o = 32; o > 0; o >>= 1) h += __shfl_xor(h, o);
    if ((threadIdx.x & 63) == 0) atomicAdd(out, (unsigned long long)h);
}

Err launch_pattern_hash(int n, int64_t nnz, const int32_t* cp, const int32_t* ri,
                        unsigned long long* out, hipStream_t st)
{
    DIAF_HIP_TRY(hipMemsetAsync(out, 0, sizeof(unsigned long long), st));
    hipLaunchKernelGGL(pattern_hash_kernel, dim3(1024), dim3(256), 0, st, n, nnz, cp, ri, out);
    DIAF_HIP_TRY(hipGetLastError());
    return {};
}

}  // namespace diaf
