// Shared device/host helpers of the HIP library: scalar traits for double
// and complex double, launch checks, and the internal interfaces between the
// API layer (diaf_api.cpp) and the kernel files.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "../../include/diaf.h"

// ---------------------------------------------------------------------------
// Complex double with the few operators the kernels need.
// ---------------------------------------------------------------------------
struct zc {
    double x, y;
};

__host__ __device__ inline zc operator+(zc a, zc b) { return {a.x + b.x, a.y + b.y}; }
__host__ __device__ inline zc operator-(zc a, zc b) { return {a.x - b.x, a.y - b.y}; }
__host__ __device__ inline zc operator-(zc a) { return {-a.x, -a.y}; }
__host__ __device__ inline zc operator*(zc a, zc b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
__host__ __device__ inline zc operator*(double s, zc a) { return {s * a.x, s * a.y}; }
__host__ __device__ inline zc operator*(zc a, double s) { return {s * a.x, s * a.y}; }
__host__ __device__ inline zc& operator+=(zc& a, zc b) { a.x += b.x; a.y += b.y; return a; }
__host__ __device__ inline zc& operator-=(zc& a, zc b) { a.x -= b.x; a.y -= b.y; return a; }

template <class T>
struct num;

template <>
struct num<double> {
    static constexpr bool is_complex = false;
    __host__ __device__ static double zero() { return 0.0; }
    __host__ __device__ static double one() { return 1.0; }
    __host__ __device__ static double mk(double r) { return r; }
    __host__ __device__ static double conj(double a) { return a; }
    __host__ __device__ static double re(double a) { return a; }
    __host__ __device__ static double im(double) { return 0.0; }
    __host__ __device__ static double abs2(double a) { return a * a; }
    __host__ __device__ static double abs(double a) { return fabs(a); }
    // conj(a) * b
    __host__ __device__ static double cmul(double a, double b) { return a * b; }
    __host__ __device__ static double div(double a, double s) { return a / s; }
    __host__ __device__ static bool finite(double a) { return isfinite(a); }
    __host__ __device__ static bool iszero(double a) { return a == 0.0; }
};

template <>
struct num<zc> {
    static constexpr bool is_complex = true;
    __host__ __device__ static zc zero() { return {0.0, 0.0}; }
    __host__ __device__ static zc one() { return {1.0, 0.0}; }
    __host__ __device__ static zc mk(double r) { return {r, 0.0}; }
    __host__ __device__ static zc conj(zc a) { return {a.x, -a.y}; }
    __host__ __device__ static double re(zc a) { return a.x; }
    __host__ __device__ static double im(zc a) { return a.y; }
    __host__ __device__ static double abs2(zc a) { return a.x * a.x + a.y * a.y; }
    // modulus without spurious overflow/underflow
    __host__ __device__ static double abs(zc a) {
        double p = fabs(a.x), q = fabs(a.y);
        double mx = p > q ? p : q, mn = p > q ? q : p;
        if (mx == 0.0) return 0.0;
        double r = mn / mx;
        return mx * sqrt(1.0 + r * r);
    }
    __host__ __device__ static zc cmul(zc a, zc b) {
        return {a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x};
    }
    __host__ __device__ static zc div(zc a, double s) { return {a.x / s, a.y / s}; }
    __host__ __device__ static bool finite(zc a) { return isfinite(a.x) && isfinite(a.y); }
    __host__ __device__ static bool iszero(zc a) { return a.x == 0.0 && a.y == 0.0; }
};

// Unit-modulus conj(z)/|z| (z != 0), scaled first so tiny entries do not
// underflow.
__host__ __device__ inline double unit_conj_phase(double z) { return z > 0.0 ? 1.0 : -1.0; }
__host__ __device__ inline zc unit_conj_phase(zc z) {
    double s = fmax(fabs(z.x), fabs(z.y));
    zc u{z.x / s, z.y / s};
    double a = sqrt(u.x * u.x + u.y * u.y);
    return {u.x / a, -u.y / a};
}

// ---------------------------------------------------------------------------
// Internal interfaces.
// ---------------------------------------------------------------------------
namespace diaf {

struct Err {
    diaf_status code = DIAF_OK;
    std::string msg;
};

#define DIAF_HIP_TRY(expr)                                                              \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess) {                                                        \
            return diaf::Err{DIAF_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)}; \
        }                                                                              \
    } while (0)

#define DIAF_TRY(expr)                 \
    do {                               \
        diaf::Err e_ = (expr);         \
        if (e_.code != DIAF_OK) return e_; \
    } while (0)

// V pattern rules as seen by the kernels.
enum VRule { V_EXPLICIT = 0, V_DIAG = 1, V_GS_UPPER = 2, V_GS_LOWER = 3, V_TOPK_UPPER = 4,
             V_TOPK_LOWER = 5, V_LEV_UPPER = 6, V_LEV_LOWER = 7, V_TOPK_BLOCK = 9 };

// Everything the factor kernels need about one launch.
template <class T>
struct FactorArgs {
    int n;
    const int32_t* Acp;
    const int32_t* Ari;
    const T* Aval;
    const int32_t* Jcp;
    const int32_t* Jri;
    const int32_t* cols;   // columns handled by this launch
    int ncols;
    int mode;              // 0 unit-norm v, 1 unit-norm w
    int vrule, vcount, lmax;
    const int32_t* Vcp_in;
    const int32_t* Vri_in;
    const int32_t* vblk;   // V_TOPK_BLOCK: rows vblk[2j] .. vblk[2j+1]-1 form j's block
    int gram_fp32;
    double stab_r, stab_tol;  // constrained v_jj of Section 3.2 (stab_r = 0: off)
    // outputs
    T* Wval;
    int32_t* Vrows;  // n * lmax, -1 padded, sorted by row
    T* Vvals;
    double* rcol;
    double* bnorm;   // ||A(:, J_j)||_F
    uint32_t* flags;
    int32_t* lcount;
};

#ifdef __HIPCC__
// Whole-wave reductions and scans over the 64 lanes by DPP moves within rows
// of 16 lanes and readlane across rows: no LDS traffic, unlike shuffles
// (ds_bpermute).  Every lane must be active.  The sums associate the same
// way on every lane (pairs, quads, half rows, rows, then the four row sums),
// so the result is the same on all lanes and for every launch.
template <int CTRL>
__device__ inline double dpp_move(double x)
{
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

__device__ inline double readlane_f64(double x, int l)
{
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readlane((int)b, l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// DPP controls: quad_perm [1,0,3,2] and [2,3,0,1], row_half_mirror,
// row_mirror, row_shr:n, row_bcast:15 and row_bcast:31.
enum : int { DPP_QXOR1 = 0xB1, DPP_QXOR2 = 0x4E, DPP_HMIRROR = 0x141, DPP_MIRROR = 0x140,
             DPP_SHR = 0x110, DPP_BCAST15 = 0x142, DPP_BCAST31 = 0x143 };

__device__ inline double dpp_wave_sum(double x)
{
    x += dpp_move<DPP_QXOR1>(x);
    x += dpp_move<DPP_QXOR2>(x);
    x += dpp_move<DPP_HMIRROR>(x);
    x += dpp_move<DPP_MIRROR>(x);
    return (readlane_f64(x, 0) + readlane_f64(x, 16)) + (readlane_f64(x, 32) + readlane_f64(x, 48));
}

__device__ inline double dpp_wave_max(double x)
{
    x = fmax(x, dpp_move<DPP_QXOR1>(x));
    x = fmax(x, dpp_move<DPP_QXOR2>(x));
    x = fmax(x, dpp_move<DPP_HMIRROR>(x));
    x = fmax(x, dpp_move<DPP_MIRROR>(x));
    return fmax(fmax(readlane_f64(x, 0), readlane_f64(x, 16)),
                fmax(readlane_f64(x, 32), readlane_f64(x, 48)));
}

__device__ inline int dpp_wave_min(int x)
{
    x = min(x, __builtin_amdgcn_update_dpp(0, x, DPP_QXOR1, 0xf, 0xf, false));
    x = min(x, __builtin_amdgcn_update_dpp(0, x, DPP_QXOR2, 0xf, 0xf, false));
    x = min(x, __builtin_amdgcn_update_dpp(0, x, DPP_HMIRROR, 0xf, 0xf, false));
    x = min(x, __builtin_amdgcn_update_dpp(0, x, DPP_MIRROR, 0xf, 0xf, false));
    return min(min(__builtin_amdgcn_readlane(x, 0), __builtin_amdgcn_readlane(x, 16)),
               min(__builtin_amdgcn_readlane(x, 32), __builtin_amdgcn_readlane(x, 48)));
}

// Inclusive prefix sum over the lanes: shifts by 1, 2, 4, 8 within each row
// (lanes shifted in from outside the row add 0), then the end of row 0 to
// rows 1 and 3 and the end of row 1 to rows 2 and 3.
__device__ inline int dpp_wave_incl_scan(int x)
{
    x += __builtin_amdgcn_update_dpp(0, x, DPP_SHR + 1, 0xf, 0xf, false);
    x += __builtin_amdgcn_update_dpp(0, x, DPP_SHR + 2, 0xf, 0xf, false);
    x += __builtin_amdgcn_update_dpp(0, x, DPP_SHR + 4, 0xf, 0xf, false);
    x += __builtin_amdgcn_update_dpp(0, x, DPP_SHR + 8, 0xf, 0xf, false);
    x += __builtin_amdgcn_update_dpp(0, x, DPP_BCAST15, 0xa, 0xf, false);
    x += __builtin_amdgcn_update_dpp(0, x, DPP_BCAST31, 0xc, 0xf, false);
    return x;
}

// Value of lane ^ 32 (the other half of the wave) by gfx950's
// v_permlane32_swap, which swaps the upper half of its first operand with
// the lower half of its second: with both operands x, the second result
// holds x of the upper half in the lower lanes and the first result x of
// the lower half in the upper lanes.  No LDS, unlike a shuffle.
__device__ inline unsigned xor32_u32(unsigned x, bool low_half)
{
    const auto r = __builtin_amdgcn_permlane32_swap(x, x, false, false);
    return low_half ? r[1] : r[0];
}

__device__ inline double xor32_f64(double x)
{
    const bool low = (threadIdx.x & 63u) < 32u;
    const long long b = __double_as_longlong(x);
    const unsigned lo = xor32_u32((unsigned)b, low), hi = xor32_u32((unsigned)(b >> 32), low);
    return __longlong_as_double(((long long)hi << 32) | lo);
}

// Columns a one-wave kernel hands back, buffered one per lane and appended
// to the global list 64 at a time, so that a launch deferring most of its
// columns does not serialise on one counter.  The list's order is
// immaterial (it is sorted before use).
struct DeferBuf {
    int reg = 0;  // lane i: the i-th buffered column
    int n = 0;    // buffered columns (the same on every lane)
};

__device__ inline void defer_flush(DeferBuf& b, int lane, int* list, int* count)
{
    if (b.n == 0) return;
    int base = 0;
    if (lane == 0) base = atomicAdd(count, b.n);
    base = __shfl(base, 0);
    if (lane < b.n) list[base + lane] = b.reg;
    b.n = 0;
}

__device__ inline void defer_push(DeferBuf& b, int j, int lane, int* list, int* count)
{
    if (lane == b.n) b.reg = j;
    if (++b.n == 64) defer_flush(b, lane, list, count);
}
#endif

}  // namespace diaf
