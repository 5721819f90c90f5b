// C ABI of the library (include/diaf.h): contexts, validation, W-pattern
// construction, size-class bucketing and factor launches, V assembly, the
// apply M = W V^{-1} and the device-resident BiCGSTAB loop.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cmath>
#include <cstring>
#include <functional>
#include <memory>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "dcommon.h"
#include "factor_kernels.h"
#include "noalloc.h"

using namespace diaf;

struct diaf_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    int64_t opt_generic_only = 0;
    int64_t opt_mid = 1;  // the mid-size one-wave kernel for unit-norm v
    int64_t opt_batch = 8;
    int64_t opt_gate_small_diag = 1;
    int64_t opt_graph = 0;
    int64_t opt_class_table = 0;  // index into kClassTables
    int64_t opt_factor_graph = 1;  // diaf_refactor replays the factor launches as a graph
    diaf::TrsvTune trsv;
    diaf::FactorTune ftune;
    hipStream_t gstream = nullptr;  // library stream for captured solve batches
};

struct diaf_model {
    diaf_ctx* ctx = nullptr;
    float* params = nullptr;
    float* m = nullptr;
    float* v = nullptr;
    float* grad = nullptr;
    float* scratch = nullptr;
    size_t scratch_pairs = 0;
    double* loss = nullptr;
    int step = 0;
};

// The factor launches of one pass, recorded for diaf_refactor: each launch
// with its arguments (column lists, deferred lists and workspaces kept
// alive in bufs), the deferred counters with the counts of the recorded
// pass, and the graph captured from them.
struct FactorPlan {
    std::vector<std::function<diaf::Err(hipStream_t)>> launches;
    std::vector<void*> bufs;
    std::vector<std::pair<int32_t*, int32_t>> counters;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    diaf_stats stats{};  // the column and launch statistics of the recorded pass
};

struct diaf_factors {
    diaf_ctx* ctx = nullptr;
    int64_t n = 0;
    int dtype = DIAF_F64;
    int mode = 0;
    int vtri = 0;
    int lmax = 1;
    int32_t* Jcp = nullptr;
    int32_t* Jri = nullptr;
    int64_t nnzW = 0;
    void* Wval = nullptr;
    int32_t* Vcp = nullptr;
    int32_t* Vri = nullptr;
    void* Vval = nullptr;
    int64_t nnzV = 0;
    int32_t* Vrows = nullptr;
    void* Vvals = nullptr;
    double* r = nullptr;
    double* bnorm = nullptr;
    uint32_t* flags = nullptr;
    int32_t* lcount = nullptr;
    diaf_stats stats{};
    // apply structures (built on first use)
    bool apply_ready = false;
    int32_t *Wrp = nullptr, *Wci = nullptr, *Vrp = nullptr, *Vci = nullptr;
    void *Wcv = nullptr, *Vcv = nullptr, *tmp = nullptr;
    TrsvCtl* ctl = nullptr;
    // block diagonal V (vtri == 3): block bounds per column, block starts,
    // offsets of the dense LU factors, the factors and row permutations, and
    // the pattern of D for DIAF_V_BLOCK
    int nblk = 0;
    int32_t* vblk = nullptr;
    int32_t* bstart = nullptr;
    int64_t* boff = nullptr;
    int64_t lu_elems = 0;
    void* blu = nullptr;
    int32_t* bperm = nullptr;
    int32_t *vpat_cp = nullptr, *vpat_ri = nullptr;
    // left variant: W, V above are those of W A ~ V (M = V^{-1} W)
    int left = 0;
    // refactoring with the same pattern: the spec, the matrix buffers and a
    // hash of A's pattern at factor time, and the recorded factor launches
    diaf_spec spec{};
    const int32_t* src_cp = nullptr;
    const int32_t* src_ri = nullptr;
    const void* src_val = nullptr;
    int64_t src_nnz = 0;
    uint64_t pat_hash = 0;
    FactorPlan* plan = nullptr;
};

namespace {

thread_local std::string g_create_err;

diaf_status fail(diaf_ctx* ctx, const Err& e)
{
    if (ctx) ctx->err = e.msg;
    return e.code;
}

diaf_status fail(diaf_ctx* ctx, diaf_status code, const std::string& msg)
{
    if (ctx) ctx->err = msg;
    return code;
}

size_t scalar_size(int dtype) { return dtype == DIAF_C128 ? 16 : 8; }

// Device memory behind dmalloc / dfree.  A factorization and a solve
// allocate and free a few dozen buffers, and hipFree synchronizes the device
// and unmaps the block each time.  dfree instead waits for the device to be
// idle (the guarantee hipFree gives: no queued work still uses the block)
// and keeps the block; dmalloc hands a kept block of the same size class
// back without calling hipMalloc.  Size classes are multiples of 256 bytes
// up to 4 KiB, then eight per power of two (at most 12.5 % slack).  At most
// kCacheCap bytes are kept per device; beyond that, and when hipMalloc runs
// out of memory, kept blocks are released.  diaf_ctx_destroy releases the
// blocks kept for its device.
//
// Temporaries of queued work (scan and sort workspaces, row counts) take
// blocks with amalloc and give them back with afree(p, st) right after the
// last launch that uses them: the block waits on a pending list until a
// synchronization of st (sync) or of the device (dfree) has covered that
// launch, and only then joins the kept blocks.  Neither call synchronizes,
// so the queue keeps running behind the host (the runtime's stream-ordered
// pool costs up to a millisecond of host time per call at the 64^3 sizes).
constexpr size_t kCacheCap = size_t(32) << 30;

struct Pending {
    void* p;
    size_t cls;
    hipStream_t st;
};

struct MemCache {
    std::mutex mu;
    std::unordered_map<void*, size_t> live;               // block -> size class
    std::unordered_map<size_t, std::vector<void*>> kept;  // size class -> idle blocks
    std::vector<Pending> pending;                         // freed, maybe still in use
    size_t kept_bytes = 0;
};

MemCache& mem_cache(int dev)
{
    static MemCache caches[64];
    return caches[dev & 63];
}

size_t size_class(size_t b)
{
    if (b <= 4096) return (b + 255) & ~size_t(255);
    const int lg = 63 - __builtin_clzll((unsigned long long)(b - 1));  // 2^lg < b <= 2^(lg+1)
    const size_t step = size_t(1) << (lg - 3);
    return (b + step - 1) / step * step;
}

int current_device()
{
    int dev = 0;
    (void)hipGetDevice(&dev);
    return dev;
}

// Pending blocks whose stream is st (all of them when all is set) join the
// kept blocks, or go back to the driver beyond kCacheCap.  The caller has
// synchronized st (the device).
void reclaim(int dev, hipStream_t st, bool all)
{
    MemCache& c = mem_cache(dev);
    std::vector<void*> drop;
    {
        std::lock_guard<std::mutex> g(c.mu);
        size_t w = 0;
        for (size_t q = 0; q < c.pending.size(); ++q) {
            const Pending& e = c.pending[q];
            if (!all && e.st != st) {
                c.pending[w++] = e;
                continue;
            }
            if (c.kept_bytes + e.cls <= kCacheCap) {
                c.kept[e.cls].push_back(e.p);
                c.kept_bytes += e.cls;
            } else {
                drop.push_back(e.p);
            }
        }
        c.pending.resize(w);
    }
    for (void* q : drop) (void)hipFree(q);
}

void release_kept(int dev)
{
    MemCache& c = mem_cache(dev);
    (void)hipDeviceSynchronize();
    reclaim(dev, nullptr, true);
    std::vector<void*> blocks;
    {
        std::lock_guard<std::mutex> g(c.mu);
        for (auto& kv : c.kept)
            for (void* q : kv.second) blocks.push_back(q);
        c.kept.clear();
        c.kept_bytes = 0;
    }
    for (void* q : blocks) (void)hipFree(q);
}

template <class P>
Err dmalloc(P** p, size_t bytes)
{
    if (bytes == 0) bytes = 16;
    const size_t cls = size_class(bytes);
    const int dev = current_device();
    MemCache& c = mem_cache(dev);
    {
        std::lock_guard<std::mutex> g(c.mu);
        auto it = c.kept.find(cls);
        if (it != c.kept.end() && !it->second.empty()) {
            void* q = it->second.back();
            it->second.pop_back();
            c.kept_bytes -= cls;
            c.live[q] = cls;
            *p = (P*)q;
            return {};
        }
    }
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, cls);
    if (e == hipErrorOutOfMemory) {
        (void)hipGetLastError();
        release_kept(dev);
        e = hipMalloc(&q, cls);
    }
    if (e != hipSuccess) return {DIAF_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e)};
    {
        std::lock_guard<std::mutex> g(c.mu);
        c.live[q] = cls;
    }
    *p = (P*)q;
    return {};
}

void dfree(void* p)
{
    if (!p) return;
    MemCache& c = mem_cache(current_device());
    size_t cls = 0;
    {
        std::lock_guard<std::mutex> g(c.mu);
        auto it = c.live.find(p);
        if (it == c.live.end()) {
            (void)hipFree(p);
            return;
        }
        cls = it->second;
        c.live.erase(it);
    }
    (void)hipDeviceSynchronize();
    reclaim(current_device(), nullptr, true);
    {
        std::lock_guard<std::mutex> g(c.mu);
        if (c.kept_bytes + cls <= kCacheCap) {
            c.kept[cls].push_back(p);
            c.kept_bytes += cls;
            return;
        }
    }
    (void)hipFree(p);
}

// Device blocks freed when the scope ends, on every return path; release()
// keeps a block whose ownership moved elsewhere.
struct DevBlocks {
    std::vector<void*> p;
    ~DevBlocks() { for (void* q : p) dfree(q); }
    void keep(void* q) { p.push_back(q); }
    void release(void* q)
    {
        for (void*& r : p)
            if (r == q) r = nullptr;
    }
};

}  // namespace

Err diaf::amalloc(void** p, size_t bytes, hipStream_t)
{
    return dmalloc(p, bytes);
}

void diaf::afree(void* p, hipStream_t st)
{
    if (!p) return;
    MemCache& c = mem_cache(current_device());
    std::lock_guard<std::mutex> g(c.mu);
    auto it = c.live.find(p);
    if (it == c.live.end()) return;  // not a block of this cache
    c.pending.push_back({p, it->second, st});
    c.live.erase(it);
}

namespace {


Err sync(hipStream_t st)
{
    DIAF_HIP_TRY(hipStreamSynchronize(st));
    reclaim(current_device(), st, false);
    return {};
}

template <class T>
Err read1(const T* dev, T* host, hipStream_t st)
{
    DIAF_HIP_TRY(hipMemcpyAsync(host, dev, sizeof(T), hipMemcpyDeviceToHost, st));
    return sync(st);
}

const char* validate_msg(int code)
{
    switch (code) {
    case 1: return "colptr not monotone or negative";
    case 2: return "row index out of range";
    case 3: return "row indices unsorted or duplicated within a column";
    case 4: return "diagonal entry missing";
    case 5: return "non-finite value";
    default: return "invalid";
    }
}

Err check_csc_host(const diaf_csc* A)
{
    if (!A) return {DIAF_EINVAL, "A is NULL"};
    if (A->n < 0 || A->n > (int64_t)INT32_MAX - 1) return {DIAF_EINVAL, "n out of range"};
    if (A->nnz < 0 || A->nnz > (int64_t)INT32_MAX) return {DIAF_EINVAL, "nnz out of range"};
    if (A->dtype != DIAF_F64 && A->dtype != DIAF_C128) return {DIAF_EINVAL, "bad dtype"};
    if (A->n > 0 && (!A->colptr || !A->rowidx || !A->val)) return {DIAF_EINVAL, "NULL array in A"};
    return {};
}

template <class T>
Err validate_A(const diaf_csc* A, hipStream_t st)
{
    int n = (int)A->n;
    if (n == 0) return {};
    int32_t* bad = nullptr;
    DIAF_TRY(dmalloc(&bad, sizeof(int32_t)));
    int32_t big = 1 << 30;
    DIAF_HIP_TRY(hipMemcpyAsync(bad, &big, sizeof(int32_t), hipMemcpyHostToDevice, st));
    // colptr[0] == 0 and colptr[n] == nnz
    int32_t ends[2];
    DIAF_HIP_TRY(hipMemcpyAsync(&ends[0], A->colptr, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    DIAF_HIP_TRY(hipMemcpyAsync(&ends[1], A->colptr + n, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    Err e = launch_validate_csc<T>(n, A->colptr, A->rowidx, (const T*)A->val, bad, st);
    int32_t code = 0;
    if (e.code == DIAF_OK) e = read1(bad, &code, st);
    dfree(bad);
    if (e.code != DIAF_OK) return e;
    if (ends[0] != 0 || ends[1] != A->nnz) return {DIAF_EINVAL, "colptr[0] != 0 or colptr[n] != nnz"};
    if (code != (1 << 30)) return {DIAF_EINVAL, std::string("A: ") + validate_msg(code)};
    return {};
}

Err validate_pattern(const diaf_pattern* P, int64_t n, int need_diag, const char* what,
                     hipStream_t st)
{
    if (!P) return {DIAF_EINVAL, std::string(what) + " is NULL"};
    if (P->n != n) return {DIAF_EINVAL, std::string(what) + ": size differs from A"};
    if (n == 0) return {};
    if (!P->colptr || (!P->rowidx && P->nnz > 0)) return {DIAF_EINVAL, std::string(what) + ": NULL array"};
    int32_t* bad = nullptr;
    DIAF_TRY(dmalloc(&bad, sizeof(int32_t)));
    int32_t big = 1 << 30;
    DIAF_HIP_TRY(hipMemcpyAsync(bad, &big, sizeof(int32_t), hipMemcpyHostToDevice, st));
    int32_t ends[2];
    DIAF_HIP_TRY(hipMemcpyAsync(&ends[0], P->colptr, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    DIAF_HIP_TRY(hipMemcpyAsync(&ends[1], P->colptr + n, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    Err e = launch_validate_pattern((int)n, P->colptr, P->rowidx, need_diag, bad, st);
    int32_t code = 0;
    if (e.code == DIAF_OK) e = read1(bad, &code, st);
    dfree(bad);
    if (e.code != DIAF_OK) return e;
    if (ends[0] != 0 || ends[1] != P->nnz) return {DIAF_EINVAL, std::string(what) + ": colptr ends"};
    if (code != (1 << 30)) return {DIAF_EINVAL, std::string(what) + ": " + validate_msg(code)};
    return {};
}

Err check_sparsify(const diaf_sparsify* sp)
{
    if (!sp) return {DIAF_EINVAL, "sparsified powers: parameters are NULL"};
    if (sp->k < 1 || sp->k > 8) return {DIAF_EINVAL, "sparsified powers: k must be in 1..8"};
    if (sp->p_i < 0 || sp->p_i > (1 << 20) || sp->p_l < 0 || sp->p_l > (1 << 20))
        return {DIAF_EINVAL, "sparsified powers: p_i and p_l must be in 0..2^20"};
    if (!(sp->tau_i >= 0.0) || !std::isfinite(sp->tau_i) || !(sp->tau_l >= 0.0) ||
        !std::isfinite(sp->tau_l))
        return {DIAF_EINVAL, "sparsified powers: tau_i and tau_l must be finite and >= 0"};
    if (sp->v0_nblocks < 0 || (sp->v0_nblocks > 0) != (sp->v0_blocks != nullptr))
        return {DIAF_EINVAL, "sparsified powers: v0_blocks must be given exactly when "
                             "v0_nblocks > 0"};
    return {};
}

// The spec checks shared by diaf_factor and diaf_autotune (host side, before
// any device work).
Err check_spec(const diaf_csc* A, const diaf_spec* spec, int mode)
{
    if (mode != DIAF_UNIT_V && mode != DIAF_UNIT_W) return {DIAF_EINVAL, "bad norm mode"};
    if (spec->v_kind < DIAF_V_EXPLICIT || spec->v_kind > DIAF_V_TOPK_BLOCK)
        return {DIAF_EINVAL, "bad v_kind"};
    const bool lev_rule = spec->v_kind == DIAF_V_LEV_UPPER || spec->v_kind == DIAF_V_LEV_LOWER;
    if (lev_rule && mode != DIAF_UNIT_V)
        return {DIAF_EINVAL, "the Section 3.1 V rule is defined for DIAF_UNIT_V"};
    if (spec->w_kind < DIAF_W_A || spec->w_kind > DIAF_W_SPARSIFIED)
        return {DIAF_EINVAL, "bad w_kind"};
    if (spec->w_kind == DIAF_W_SPARSIFIED) {
        DIAF_TRY(check_sparsify(&spec->sparsify));
    }
    if (!(spec->stab_r >= 0.0) || !std::isfinite(spec->stab_r) || !(spec->stab_tol >= 0.0) ||
        !std::isfinite(spec->stab_tol))
        return {DIAF_EINVAL, "stab_r and stab_tol must be finite and >= 0"};
    if ((spec->v_kind == DIAF_V_TOPK_UPPER || spec->v_kind == DIAF_V_TOPK_LOWER || lev_rule ||
         spec->v_kind == DIAF_V_TOPK_BLOCK) &&
        (spec->v_count < 1 || spec->v_count > 64))
        return {DIAF_EINVAL, "v_count must be in 1..64"};
    if (spec->w_kind == DIAF_W_A_1HOP_TOPK && (spec->w_topk < 0 || spec->w_topk > 256))
        return {DIAF_EINVAL, "w_topk must be in 0..256"};
    if (spec->left != 0 && spec->left != 1) return {DIAF_EINVAL, "left must be 0 or 1"};
    return {};
}

// Algorithm 1 (Section 4) with V_0 = diagonals: S built and sparsified once,
// then the per-column level expansion, counted and filled; columns that
// outgrow the small LDS tables are rerun with the large ones.
template <class T>
Err build_sparsified_t(const diaf_csc* A, const diaf_sparsify* sp, int32_t* Jcp, int32_t** Jri_out,
                       int64_t* nnz_out, bool alloc_rows, int32_t* rows_given, hipStream_t st)
{
    const int n = (int)A->n;
    const size_t nnz = (size_t)A->nnz;
    struct Free {
        std::vector<void*> p;
        ~Free() { for (void* q : p) dfree(q); }
    } fr;
    const auto take = [&](auto** ptr, size_t bytes) -> Err {
        DIAF_TRY(dmalloc(ptr, bytes > 0 ? bytes : 1));
        fr.p.push_back(*ptr);
        return {};
    };
    T* Sval = nullptr;
    int32_t *bad = nullptr, *Sri = nullptr, *scnt = nullptr, *cnt = nullptr, *lists = nullptr,
            *nover = nullptr, *rb = nullptr;
    const int32_t* Scp = A->colptr;
    const T* Aval = (const T*)A->val;
    DIAF_TRY(take(&scnt, sizeof(int32_t) * (size_t)n));
    DIAF_TRY(take(&cnt, sizeof(int32_t) * (size_t)(n + 1)));
    DIAF_TRY(take(&lists, sizeof(int32_t) * 2 * (size_t)n));  // deferred, then failed columns
    DIAF_TRY(take(&bad, sizeof(int32_t) * 3));  // bad flags, #deferred, #failed
    nover = bad + 1;
    int32_t* deferred = lists;
    int32_t* failed = lists + n;
    DIAF_HIP_TRY(hipMemsetAsync(bad, 0, sizeof(int32_t) * 3, st));
    if (sp->v0_nblocks == 0) {
        // V_0 the diagonal matrices: S in A's column layout
        T* d = nullptr;
        DIAF_TRY(take(&d, sizeof(T) * (size_t)n));
        DIAF_TRY(take(&Sval, sizeof(T) * nnz));
        DIAF_TRY(take(&Sri, sizeof(int32_t) * nnz));
        DIAF_TRY(launch_sp_diag<T>(n, A->colptr, A->rowidx, Aval, d, bad, st));
        DIAF_TRY(launch_sp_build_s<T>(n, A->colptr, A->rowidx, Aval, d, sp->tau_i, sp->p_i, Sri,
                                      Sval, scnt, bad, st));
        int32_t flags = 0;
        DIAF_TRY(read1(bad, &flags, st));
        if (flags & 1)
            return {DIAF_EINVAL,
                    "sparsified powers: A has a zero diagonal entry (D^{-1} undefined)"};
        if (flags & 2)
            return {DIAF_EUNSUPPORTED,
                    "sparsified powers: a column of A has more than 1024 entries"};
    } else {
        // V_0 block diagonal: the blocks, A's block diagonal part D, its LU
        const int nb = sp->v0_nblocks;
        std::vector<int32_t> s(nb + 1);
        DIAF_HIP_TRY(hipMemcpyAsync(s.data(), sp->v0_blocks, sizeof(int32_t) * (nb + 1),
                                    hipMemcpyDeviceToHost, st));
        DIAF_TRY(sync(st));
        if (s[0] != 0 || s[nb] != n)
            return {DIAF_EINVAL, "sparsified powers: the V_0 block starts must run from 0 to n"};
        std::vector<int32_t> bounds(2 * (size_t)n), bidh(n);
        std::vector<int64_t> off(nb + 1, 0);
        for (int b = 0; b < nb; ++b) {
            const int sz = s[b + 1] - s[b];
            if (sz <= 0)
                return {DIAF_EINVAL, "sparsified powers: the V_0 block starts must increase"};
            if (sz > 64)
                return {DIAF_EUNSUPPORTED, "sparsified powers: V_0 blocks of at most 64 rows"};
            for (int j = s[b]; j < s[b + 1]; ++j) {
                bounds[2 * (size_t)j] = s[b];
                bounds[2 * (size_t)j + 1] = s[b + 1];
                bidh[j] = b;
            }
            off[b + 1] = off[b] + (int64_t)sz * sz;
        }
        int32_t *bid = nullptr, *bstart = nullptr, *Dcp = nullptr, *Dri = nullptr, *perm = nullptr;
        int64_t* boff = nullptr;
        T *Dval = nullptr, *LU = nullptr;
        DIAF_TRY(take(&rb, sizeof(int32_t) * bounds.size()));
        DIAF_TRY(take(&bid, sizeof(int32_t) * (size_t)n));
        DIAF_TRY(take(&bstart, sizeof(int32_t) * (nb + 1)));
        DIAF_TRY(take(&boff, sizeof(int64_t) * (nb + 1)));
        DIAF_HIP_TRY(hipMemcpyAsync(rb, bounds.data(), sizeof(int32_t) * bounds.size(),
                                    hipMemcpyHostToDevice, st));
        DIAF_HIP_TRY(hipMemcpyAsync(bid, bidh.data(), sizeof(int32_t) * (size_t)n,
                                    hipMemcpyHostToDevice, st));
        DIAF_HIP_TRY(hipMemcpyAsync(bstart, s.data(), sizeof(int32_t) * (nb + 1),
                                    hipMemcpyHostToDevice, st));
        DIAF_HIP_TRY(hipMemcpyAsync(boff, off.data(), sizeof(int64_t) * (nb + 1),
                                    hipMemcpyHostToDevice, st));
        DIAF_TRY(take(&Dcp, sizeof(int32_t) * (size_t)(n + 1)));
        DIAF_TRY(launch_sp_block_d<T>(n, A->colptr, A->rowidx, Aval, rb, cnt, nullptr, nullptr,
                                      nullptr, st));
        DIAF_TRY(exclusive_scan_i32(cnt, Dcp, n, st));
        int32_t dn = 0;
        DIAF_TRY(read1(Dcp + n, &dn, st));
        DIAF_TRY(take(&Dri, sizeof(int32_t) * (size_t)dn));
        DIAF_TRY(take(&Dval, sizeof(T) * (size_t)dn));
        DIAF_TRY(launch_sp_block_d<T>(n, A->colptr, A->rowidx, Aval, rb, nullptr, Dcp, Dri, Dval,
                                      st));
        DIAF_TRY(take(&LU, sizeof(T) * (size_t)off[nb]));
        DIAF_TRY(take(&perm, sizeof(int32_t) * (size_t)n));
        DIAF_TRY(launch_block_lu<T>(nb, bstart, boff, Dcp, Dri, Dval, LU, perm, bad, st));
        int32_t nsing = 0;
        DIAF_TRY(read1(bad, &nsing, st));
        if (nsing & ((1 << 30) - 1))
            return {DIAF_EINVAL, "sparsified powers: a diagonal block of A (V_0) is singular"};
        DIAF_HIP_TRY(hipMemsetAsync(bad, 0, sizeof(int32_t), st));
        // S: count, layout, fill
        int32_t* Scp_own = nullptr;
        DIAF_TRY(take(&Scp_own, sizeof(int32_t) * (size_t)(n + 1)));
        DIAF_TRY(launch_sp_build_s_block<T>(n, A->colptr, A->rowidx, Aval, rb, bid, bstart, boff,
                                            LU, perm, sp->tau_i, sp->p_i, scnt, nullptr, nullptr,
                                            nullptr, bad, st));
        int32_t flags = 0;
        DIAF_TRY(read1(bad, &flags, st));
        if (flags & 2)
            return {DIAF_EUNSUPPORTED, "sparsified powers: a column of A, or of S before "
                                       "dropping, has more than 1024 entries"};
        DIAF_TRY(exclusive_scan_i32(scnt, Scp_own, n, st));
        int32_t sn = 0;
        DIAF_TRY(read1(Scp_own + n, &sn, st));
        DIAF_TRY(take(&Sri, sizeof(int32_t) * (size_t)sn));
        DIAF_TRY(take(&Sval, sizeof(T) * (size_t)sn));
        DIAF_TRY(launch_sp_build_s_block<T>(n, A->colptr, A->rowidx, Aval, rb, bid, bstart, boff,
                                            LU, perm, sp->tau_i, sp->p_i, scnt, Scp_own, Sri,
                                            Sval, bad, st));
        Scp = Scp_own;
    }
    DIAF_TRY(launch_sp_expand<T>(n, Scp, Sri, Sval, scnt, sp->k, sp->tau_l, sp->p_l, rb, nullptr,
                                 n, 0, cnt, nullptr, nullptr, deferred, nover, st));
    int32_t ndef = 0;
    DIAF_TRY(read1(nover, &ndef, st));
    if (ndef > 0) {
        DIAF_TRY(launch_sp_expand<T>(n, Scp, Sri, Sval, scnt, sp->k, sp->tau_l, sp->p_l, rb,
                                     deferred, ndef, 1, cnt, nullptr, nullptr, failed, nover + 1,
                                     st));
        int32_t nfail = 0;
        DIAF_TRY(read1(nover + 1, &nfail, st));
        if (nfail > 0)
            return {DIAF_EUNSUPPORTED, SpCaps<T>::TL == 2048
                                           ? "sparsified powers: a power vector exceeds 2048 "
                                             "rows or a pattern 4096 rows"
                                           : "sparsified powers: a power vector exceeds 1024 "
                                             "rows or a pattern 2048 rows (complex)"};
    }
    DIAF_TRY(exclusive_scan_i32(cnt, Jcp, n, st));
    int32_t tot = 0;
    DIAF_TRY(read1(Jcp + n, &tot, st));
    *nnz_out = tot;
    int32_t* rows = rows_given;
    if (!rows && alloc_rows) {
        DIAF_TRY(dmalloc(Jri_out, sizeof(int32_t) * (size_t)(tot > 0 ? tot : 1)));
        rows = *Jri_out;
    }
    if (rows) {
        DIAF_TRY(launch_sp_expand<T>(n, Scp, Sri, Sval, scnt, sp->k, sp->tau_l, sp->p_l, rb,
                                     nullptr, n, 0, nullptr, Jcp, rows, nullptr, nullptr, st));
        DIAF_TRY(launch_sp_expand<T>(n, Scp, Sri, Sval, scnt, sp->k, sp->tau_l, sp->p_l, rb,
                                     deferred, ndef, 1, nullptr, Jcp, rows, nullptr, nullptr, st));
    }
    DIAF_TRY(sync(st));
    return {};
}

Err build_sparsified(const diaf_csc* A, const diaf_sparsify* sp, int32_t* Jcp, int32_t** Jri_out,
                     int64_t* nnz_out, bool alloc_rows, int32_t* rows_given, hipStream_t st)
{
    DIAF_TRY(check_sparsify(sp));
    return A->dtype == DIAF_F64
               ? build_sparsified_t<double>(A, sp, Jcp, Jri_out, nnz_out, alloc_rows, rows_given,
                                            st)
               : build_sparsified_t<zc>(A, sp, Jcp, Jri_out, nnz_out, alloc_rows, rows_given, st);
}

// Builds the W pattern (colptr, rowidx allocated here unless provided).
template <class T>
Err build_pattern(const diaf_csc* A, int w_kind, int w_topk, int32_t* Jcp, int32_t** Jri_out,
                  int64_t* nnz_out, bool alloc_rows, int32_t* rows_given, hipStream_t st,
                  const diaf_sparsify* sp = nullptr)
{
    const int n = (int)A->n;
    if (w_kind == DIAF_W_SPARSIFIED)
        return build_sparsified(A, sp, Jcp, Jri_out, nnz_out, alloc_rows, rows_given, st);
    if (w_kind == DIAF_W_A) {
        DIAF_HIP_TRY(hipMemcpyAsync(Jcp, A->colptr, sizeof(int32_t) * (n + 1),
                                    hipMemcpyDeviceToDevice, st));
        *nnz_out = A->nnz;
        if (rows_given) {
            DIAF_HIP_TRY(hipMemcpyAsync(rows_given, A->rowidx, sizeof(int32_t) * A->nnz,
                                        hipMemcpyDeviceToDevice, st));
        } else if (alloc_rows) {
            DIAF_TRY(dmalloc(Jri_out, sizeof(int32_t) * A->nnz));
            DIAF_HIP_TRY(hipMemcpyAsync(*Jri_out, A->rowidx, sizeof(int32_t) * A->nnz,
                                        hipMemcpyDeviceToDevice, st));
        }
        return {};
    }
    if (w_kind == DIAF_W_ALG2_DIAG || w_kind == DIAF_W_ALG2_GS_UPPER ||
        w_kind == DIAF_W_ALG2_GS_LOWER) {
        // Algorithm 2: column j of W has the pattern of A^* v_j for a generic
        // v_j in V_0, i.e. the union of the rows of A at the pattern of
        // column j of V_0 (the union pattern with V_0 as the outer lists and
        // the rows of A, from its CSR copy, as the inner lists)
        const int v0 = w_kind - DIAF_W_ALG2_DIAG;
        int32_t *vcnt = nullptr, *Vcp = nullptr, *Vri = nullptr, *rp = nullptr, *ci = nullptr;
        int32_t *cnt = nullptr, *mx = nullptr;
        T* cv = nullptr;
        struct Free {
            std::vector<void*> p;
            ~Free() { for (void* q : p) dfree(q); }
        } fr;
        DIAF_TRY(dmalloc(&vcnt, sizeof(int32_t) * (n + 1)));
        fr.p.push_back(vcnt);
        DIAF_TRY(dmalloc(&Vcp, sizeof(int32_t) * (n + 1)));
        fr.p.push_back(Vcp);
        DIAF_TRY(launch_v0_pattern(n, A->colptr, A->rowidx, v0, vcnt, nullptr, nullptr, st));
        DIAF_TRY(exclusive_scan_i32(vcnt, Vcp, n, st));
        int32_t nv = 0;
        DIAF_TRY(read1(Vcp + n, &nv, st));
        DIAF_TRY(dmalloc(&Vri, sizeof(int32_t) * (size_t)(nv > 0 ? nv : 1)));
        fr.p.push_back(Vri);
        DIAF_TRY(launch_v0_pattern(n, A->colptr, A->rowidx, v0, nullptr, Vcp, Vri, st));
        DIAF_TRY(dmalloc(&rp, sizeof(int32_t) * (n + 1)));
        fr.p.push_back(rp);
        DIAF_TRY(dmalloc(&ci, sizeof(int32_t) * (size_t)A->nnz));
        fr.p.push_back(ci);
        DIAF_TRY(dmalloc(&cv, sizeof(T) * (size_t)A->nnz));
        fr.p.push_back(cv);
        DIAF_TRY(csc_to_csr<T>(n, A->nnz, A->colptr, A->rowidx, (const T*)A->val, rp, ci, cv, st));
        DIAF_TRY(dmalloc(&cnt, sizeof(int32_t) * (n + 1)));
        fr.p.push_back(cnt);
        DIAF_TRY(dmalloc(&mx, sizeof(int32_t)));
        fr.p.push_back(mx);
        DIAF_HIP_TRY(hipMemsetAsync(mx, 0, sizeof(int32_t), st));
        DIAF_TRY(launch_cand_count(n, Vcp, Vri, rp, cnt, mx, st));
        int32_t maxcand = 0;
        DIAF_TRY(read1(mx, &maxcand, st));
        DIAF_TRY(launch_pattern_a2(n, Vcp, Vri, rp, ci, maxcand, cnt, nullptr, nullptr, st));
        DIAF_TRY(exclusive_scan_i32(cnt, Jcp, n, st));
        int32_t tot = 0;
        DIAF_TRY(read1(Jcp + n, &tot, st));
        *nnz_out = tot;
        int32_t* rows = rows_given;
        if (!rows && alloc_rows) {
            DIAF_TRY(dmalloc(Jri_out, sizeof(int32_t) * (size_t)(tot > 0 ? tot : 1)));
            rows = *Jri_out;
        }
        if (rows) DIAF_TRY(launch_pattern_a2(n, Vcp, Vri, rp, ci, maxcand, nullptr, Jcp, rows, st));
        DIAF_TRY(sync(st));
        return {};
    }
    if (w_kind != DIAF_W_A2 && w_kind != DIAF_W_A_1HOP_TOPK)
        return {DIAF_EINVAL, "pattern kind not buildable here"};
    int32_t *cnt = nullptr, *mx = nullptr;
    DIAF_TRY(dmalloc(&cnt, sizeof(int32_t) * (n + 1)));
    DIAF_TRY(dmalloc(&mx, sizeof(int32_t)));
    DIAF_HIP_TRY(hipMemsetAsync(mx, 0, sizeof(int32_t), st));
    DIAF_TRY(launch_cand_count(n, A->colptr, A->rowidx, A->colptr, cnt, mx, st));
    int32_t maxcand = 0;
    DIAF_TRY(read1(mx, &maxcand, st));
    // 1-hop rule: columns grouped by their number of two-hop candidates, so
    // each launch sizes its LDS for its own class, not for the largest
    // column; the grouping is a class sort on the device (as for the factor
    // launches), and only the class counts come back to the host
    struct HopClass { int cand_max; int count; const int32_t* cols; };
    std::vector<HopClass> hop;
    int32_t *hsorted = nullptr, *hmeta = nullptr;
    struct HopFree {
        int32_t** a; int32_t** b;
        ~HopFree() { dfree(*a); dfree(*b); }
    } hopfree{&hsorted, &hmeta};
    if (w_kind == DIAF_W_A_1HOP_TOPK) {
        ColumnClasses hc{};
        const int bounds[] = {256, 512, 1024, 2048, 4096};
        hc.ncls = 5;
        for (int c = 0; c < hc.ncls; ++c) hc.kcap[c] = hc.tcap[c] = bounds[c] - w_topk - 1;
        DIAF_TRY(dmalloc(&hsorted, sizeof(int32_t) * (size_t)std::max(n, 1)));
        DIAF_TRY(dmalloc(&hmeta, sizeof(int32_t) * (ColumnClasses::kMax + 1)));
        DIAF_TRY(launch_classify_columns(n, n, nullptr, cnt, cnt, hc, hsorted, hmeta, nullptr, st));
        int32_t hm[ColumnClasses::kMax + 1] = {};
        DIAF_HIP_TRY(hipMemcpyAsync(hm, hmeta, sizeof(int32_t) * (hc.ncls + 1),
                                    hipMemcpyDeviceToHost, st));
        DIAF_TRY(sync(st));
        if (hm[hc.ncls] > 0)
            return {DIAF_EUNSUPPORTED, "1-hop pattern: too many two-hop candidates in a column"};
        int off = 0;
        for (int c = 0; c < hc.ncls; ++c) {
            if (hm[c]) hop.push_back({hc.kcap[c], hm[c], hsorted + off});
            off += hm[c];
        }
    }
    // the 1-hop rule runs once into per-column slots (capacity |A(:, j)| +
    // w_topk), which are packed after the scan of the counts
    int32_t* slots = nullptr;
    struct SlotFree {
        int32_t** p;
        ~SlotFree() { dfree(*p); }
    } slotfree{&slots};
    if (w_kind == DIAF_W_A2) {
        DIAF_TRY(launch_pattern_a2(n, A->colptr, A->rowidx, A->colptr, A->rowidx, maxcand, cnt,
                                   nullptr, nullptr, st));
    } else {
        DIAF_TRY(dmalloc(&slots, sizeof(int32_t) * ((size_t)A->nnz + (size_t)n * w_topk + 1)));
        for (auto& c : hop)
            DIAF_TRY(launch_pattern_1hop<T>(n, A->colptr, A->rowidx, (const T*)A->val, w_topk,
                                            c.cand_max, c.cols, c.count, cnt, slots, st));
    }
    DIAF_TRY(exclusive_scan_i32(cnt, Jcp, n, st));
    int32_t tot = 0;
    DIAF_TRY(read1(Jcp + n, &tot, st));
    *nnz_out = tot;
    int32_t* rows = rows_given;
    if (!rows && alloc_rows) {
        DIAF_TRY(dmalloc(Jri_out, sizeof(int32_t) * (size_t)tot));
        rows = *Jri_out;
    }
    if (rows) {
        if (w_kind == DIAF_W_A2)
            DIAF_TRY(launch_pattern_a2(n, A->colptr, A->rowidx, A->colptr, A->rowidx, maxcand,
                                       nullptr, Jcp, rows, st));
        else
            DIAF_TRY(launch_compact_slots(n, A->colptr, w_topk, cnt, slots, Jcp, rows, st));
    }
    DIAF_TRY(sync(st));
    dfree(cnt);
    dfree(mx);
    return {};
}

void free_factors(diaf_factors* F)
{
    if (!F) return;
    for (void* p : {(void*)F->Jcp, (void*)F->Jri, F->Wval, (void*)F->Vcp, (void*)F->Vri, F->Vval,
                    (void*)F->Vrows, F->Vvals, (void*)F->r, (void*)F->bnorm, (void*)F->flags,
                    (void*)F->lcount, (void*)F->Wrp, (void*)F->Wci, (void*)F->Vrp, (void*)F->Vci,
                    F->Wcv, F->Vcv, F->tmp, (void*)F->ctl, (void*)F->vblk,
                    (void*)F->bstart, (void*)F->boff, F->blu, (void*)F->bperm,
                    (void*)F->vpat_cp, (void*)F->vpat_ri})
        dfree(p);
    if (F->plan) {
        if (F->plan->exec) (void)hipGraphExecDestroy(F->plan->exec);
        if (F->plan->graph) (void)hipGraphDestroy(F->plan->graph);
        for (void* p : F->plan->bufs) dfree(p);
        delete F->plan;
    }
    delete F;
}

int vtri_of(int v_kind)
{
    switch (v_kind) {
    case DIAF_V_GS_UPPER:
    case DIAF_V_TOPK_UPPER:
    case DIAF_V_LEV_UPPER: return 1;
    case DIAF_V_GS_LOWER:
    case DIAF_V_TOPK_LOWER:
    case DIAF_V_LEV_LOWER: return -1;
    case DIAF_V_DIAG: return 0;
    case DIAF_V_BLOCK:
    case DIAF_V_TOPK_BLOCK: return 3;
    default: return 2;  // determined from the explicit pattern
    }
}

// Block diagonal V: checks the block starts (0 = s_0 < s_1 < ... < s_nb = n,
// blocks of at most 64 rows) and stores the per-column bounds, the starts
// and the offsets of the dense LU factors in F.
Err setup_blocks(const diaf_spec* spec, int n, diaf_factors* F, hipStream_t st)
{
    const int nb = spec->v_nblocks;
    if (!spec->v_blocks || nb < 1 || nb > n)
        return {DIAF_EINVAL, "block V: v_blocks must hold v_nblocks + 1 starts, 1 <= v_nblocks <= n"};
    std::vector<int32_t> s(nb + 1);
    DIAF_HIP_TRY(hipMemcpyAsync(s.data(), spec->v_blocks, sizeof(int32_t) * (nb + 1),
                                hipMemcpyDeviceToHost, st));
    DIAF_TRY(sync(st));
    if (s[0] != 0 || s[nb] != n) return {DIAF_EINVAL, "block V: the starts must run from 0 to n"};
    std::vector<int32_t> bounds(2 * (size_t)n);
    std::vector<int64_t> off(nb + 1, 0);
    for (int b = 0; b < nb; ++b) {
        const int sz = s[b + 1] - s[b];
        if (sz <= 0) return {DIAF_EINVAL, "block V: the starts must increase strictly"};
        if (sz > 64) return {DIAF_EUNSUPPORTED, "block V: blocks of at most 64 rows"};
        for (int j = s[b]; j < s[b + 1]; ++j) {
            bounds[2 * (size_t)j] = s[b];
            bounds[2 * (size_t)j + 1] = s[b + 1];
        }
        off[b + 1] = off[b] + (int64_t)sz * sz;
    }
    DIAF_TRY(dmalloc(&F->vblk, sizeof(int32_t) * bounds.size()));
    DIAF_TRY(dmalloc(&F->bstart, sizeof(int32_t) * (nb + 1)));
    DIAF_TRY(dmalloc(&F->boff, sizeof(int64_t) * (nb + 1)));
    DIAF_HIP_TRY(hipMemcpyAsync(F->vblk, bounds.data(), sizeof(int32_t) * bounds.size(),
                                hipMemcpyHostToDevice, st));
    DIAF_HIP_TRY(hipMemcpyAsync(F->bstart, s.data(), sizeof(int32_t) * (nb + 1),
                                hipMemcpyHostToDevice, st));
    DIAF_HIP_TRY(hipMemcpyAsync(F->boff, off.data(), sizeof(int64_t) * (nb + 1),
                                hipMemcpyHostToDevice, st));
    DIAF_TRY(sync(st));
    F->nblk = nb;
    F->lu_elems = off[nb];
    return {};
}

// Factor the listed columns (all columns when cols is empty) into F's
// buffers, which must already be allocated.
// Size classes (|J_j| capacity, gathered-entry capacity) of the factor
// launches; a column takes the first class that holds it.  Every table has
// (32, 256) and (64, 1024) among its classes, with the classes before each of
// them inside it, so the columns that reach the one-wave and mid-size
// kernels are the same for every table; the generic kernel's results do not
// depend on the capacities either.  The autotuner picks the table.
struct ClassTable {
    int n;
    int cap[ColumnClasses::kMax][2];
};
const ClassTable kClassTables[] = {
    {7, {{16, 128}, {32, 256}, {64, 512}, {64, 1024}, {128, 2048}, {256, 4096}, {256, 8192}}},
    {8, {{16, 128}, {32, 256}, {48, 512}, {64, 1024}, {96, 2048}, {128, 3072}, {192, 4096},
         {256, 8192}}},
    {4, {{32, 256}, {64, 1024}, {128, 4096}, {256, 8192}}},
    {8, {{16, 128}, {32, 256}, {64, 512}, {64, 1024}, {128, 1536}, {128, 2048}, {192, 4096},
         {256, 8192}}},
};
constexpr int kNumClassTables = (int)(sizeof(kClassTables) / sizeof(kClassTables[0]));

// rec: when given, the factor launches are also recorded there (with the
// buffers they read kept alive) for replay by diaf_refactor.
template <class T>
Err factor_columns(diaf_ctx* ctx, const diaf_csc* A, const diaf_spec* spec, int mode,
                   diaf_factors* F, const std::vector<int32_t>* only, int* nbuckets,
                   FactorPlan* rec = nullptr)
{
    hipStream_t st = ctx->stream;
    const int n = (int)A->n;
    std::vector<void*> to_free;
    struct FreeAll {
        std::vector<void*>* v;
        ~FreeAll() { for (void* p : *v) dfree(p); }
    } free_all{&to_free};
    std::vector<void*>& keep = rec ? rec->bufs : to_free;
    const auto scratch = [&](int32_t** p, size_t count) -> Err {
        DIAF_TRY(dmalloc(p, sizeof(int32_t) * std::max<size_t>(count, 1)));
        keep.push_back(*p);
        return {};
    };
    // per-column sizes, then the columns sorted by size class on the device
    // (stable: ascending columns, or the order of `only`, within a class)
    const ClassTable& tab = kClassTables[ctx->opt_class_table];
    const int ncls = tab.n;
    ColumnClasses cc{};
    cc.ncls = ncls;
    for (int c = 0; c < ncls; ++c) { cc.kcap[c] = tab.cap[c][0]; cc.tcap[c] = tab.cap[c][1]; }
    for (int c = 0; c < ncls; ++c) {
        F->stats.class_kcap[c] = cc.kcap[c];
        F->stats.class_tcap[c] = cc.tcap[c];
    }
    const int m = only ? (int)only->size() : n;
    int32_t *kd = nullptr, *td = nullptr, *sel = nullptr, *sorted = nullptr, *meta = nullptr;
    DIAF_TRY(scratch(&kd, n));
    DIAF_TRY(scratch(&td, n));
    DIAF_TRY(scratch(&sorted, m));
    DIAF_TRY(scratch(&meta, 2 * (ColumnClasses::kMax + 1) + 2));
    DIAF_TRY(launch_column_sizes(n, A->colptr, F->Jcp, F->Jri, kd, td, st));
    if (only) {
        DIAF_TRY(scratch(&sel, m));
        DIAF_HIP_TRY(hipMemcpyAsync(sel, only->data(), sizeof(int32_t) * m, hipMemcpyHostToDevice,
                                    st));
    }
    int32_t* dmeta = meta + ColumnClasses::kMax + 1;  // counts of the deferred columns
    int32_t* maxes = meta + 2 * (ColumnClasses::kMax + 1);
    DIAF_TRY(launch_classify_columns(n, m, sel, kd, td, cc, sorted, meta, maxes, st));
    int32_t hm[2 * (ColumnClasses::kMax + 1) + 2] = {};
    DIAF_HIP_TRY(hipMemcpyAsync(hm, meta, sizeof(hm), hipMemcpyDeviceToHost, st));
    DIAF_TRY(sync(st));
    if (hm[ncls] > 0) {
        // a column beyond every class: name the first one
        std::vector<int32_t> kh(n), th(n);
        DIAF_HIP_TRY(hipMemcpyAsync(kh.data(), kd, sizeof(int32_t) * n, hipMemcpyDeviceToHost, st));
        DIAF_HIP_TRY(hipMemcpyAsync(th.data(), td, sizeof(int32_t) * n, hipMemcpyDeviceToHost, st));
        DIAF_TRY(sync(st));
        for (int q = 0; q < m; ++q) {
            const int j = only ? (*only)[q] : q;
            if (kh[j] > cc.kcap[ncls - 1] || th[j] > cc.tcap[ncls - 1])
                return {DIAF_EUNSUPPORTED, "column " + std::to_string(j) + ": |J_j| = " +
                                               std::to_string(kh[j]) + ", gathered entries = " +
                                               std::to_string(th[j]) +
                                               " exceed the limits (256, 8192)"};
        }
        return {DIAF_EINVAL, "internal: column class counts"};
    }
    // launch list: (class, first entry, count) over `sorted`
    struct Seg {
        int c;
        const int32_t* cols;
        int count;
    };
    std::vector<Seg> segs;
    {
        int off = 0;
        for (int c = 0; c < ncls; ++c) {
            if (hm[c]) segs.push_back({c, sorted + off, hm[c]});
            off += hm[c];
        }
    }
    F->stats.kmax = hm[2 * (ColumnClasses::kMax + 1)];
    F->stats.mmax = hm[2 * (ColumnClasses::kMax + 1) + 1];
    FactorArgs<T> fa{};
    fa.n = n;
    fa.Acp = A->colptr;
    fa.Ari = A->rowidx;
    fa.Aval = (const T*)A->val;
    fa.Jcp = F->Jcp;
    fa.Jri = F->Jri;
    fa.mode = mode;
    fa.vrule = spec->v_kind == DIAF_V_BLOCK ? V_EXPLICIT : spec->v_kind;
    fa.vcount = spec->v_count;
    fa.lmax = F->lmax;
    fa.Vcp_in = spec->v_explicit ? spec->v_explicit->colptr : nullptr;
    fa.Vri_in = spec->v_explicit ? spec->v_explicit->rowidx : nullptr;
    if (spec->v_kind == DIAF_V_BLOCK) {  // the pattern of D, built by factor_impl
        fa.Vcp_in = F->vpat_cp;
        fa.Vri_in = F->vpat_ri;
    }
    fa.vblk = F->vblk;
    fa.gram_fp32 = spec->gram_fp32;
    fa.stab_r = spec->stab_r;
    fa.stab_tol = spec->stab_tol;
    fa.Wval = (T*)F->Wval;
    fa.Vrows = F->Vrows;
    fa.Vvals = (T*)F->Vvals;
    fa.rcol = F->r;
    fa.bnorm = F->bnorm;
    fa.flags = F->flags;
    fa.lcount = F->lcount;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> events;
    std::vector<int> ev_class;  // -1: one-wave kernel, -2: mid-size kernel, else generic class
    struct FreeEvents {
        std::vector<std::pair<hipEvent_t, hipEvent_t>>* v;
        ~FreeEvents() {
            for (auto& e : *v) {
                (void)hipEventDestroy(e.first);
                (void)hipEventDestroy(e.second);
            }
        }
    } free_events{&events};
    // one factor launch: timed with events, and recorded for replay
    const auto timed = [&](int cls, std::function<Err(hipStream_t)> launch) -> Err {
        hipEvent_t e0 = nullptr, e1 = nullptr;
        DIAF_HIP_TRY(hipEventCreate(&e0));
        if (hipEventCreate(&e1) != hipSuccess) {
            (void)hipEventDestroy(e0);
            return {DIAF_EDEVICE, "hipEventCreate"};
        }
        events.push_back({e0, e1});
        ev_class.push_back(cls);
        DIAF_HIP_TRY(hipEventRecord(e0, st));
        DIAF_TRY(launch(st));
        DIAF_HIP_TRY(hipEventRecord(e1, st));
        if (rec) rec->launches.push_back(std::move(launch));
        return {};
    };
    // a counter cleared before its launch (by a kernel, so that a captured
    // graph holds no memset node)
    const auto clear_counter = [&](int32_t* c) -> Err {
        DIAF_HIP_TRY(hipMemsetAsync(c, 0, sizeof(int32_t), st));
        if (rec)
            rec->launches.push_back(
                [c](hipStream_t s) -> Err { return noalloc_clear(c, sizeof(int32_t), s); });
        return {};
    };
    int nb = 0;
    // Small columns (the classes within 32 rows of J_j and 256 gathered
    // entries, which come first in `sorted`) go to the one-wave kernel (both
    // norm modes); columns it cannot hold (shadow above 64 rows) come back on
    // a deferred list, sorted and classified again for the generic kernel.
    // The FP32-Gram variant is implemented by the generic kernel only.
    if (!ctx->opt_generic_only && !spec->gram_fp32 && F->lmax <= 8) {
        int nsmall = 0, nseg = 0;
        while (nseg < (int)segs.size() && cc.kcap[segs[nseg].c] <= 32 && cc.tcap[segs[nseg].c] <= 256)
            nsmall += segs[nseg++].count;
        if (nsmall > 0) {
            segs.erase(segs.begin(), segs.begin() + nseg);
            int32_t *defl = nullptr, *ndef = nullptr, *dsorted = nullptr, *dtmp = nullptr;
            DIAF_TRY(scratch(&defl, nsmall));
            DIAF_TRY(scratch(&ndef, 1));
            DIAF_TRY(clear_counter(ndef));
            fa.cols = sorted;
            fa.ncols = nsmall;
            const FactorTune tune = ctx->ftune;
            DIAF_TRY(timed(-1, [fa, defl, ndef, tune](hipStream_t s) -> Err {
                return launch_factor_small<T>(fa, defl, ndef, tune, s);
            }));
            ++nb;
            int32_t nd = 0;
            DIAF_TRY(read1(ndef, &nd, st));
            if (rec) rec->counters.push_back({ndef, nd});
            F->stats.cols_small += nsmall - nd;
            F->stats.occ_small = small_occupancy<T>(mode);
            if (nd > 0) {
                DIAF_TRY(scratch(&dtmp, nd));
                DIAF_TRY(scratch(&dsorted, nd));
                DIAF_TRY(sort_columns(n, nd, defl, dtmp, st));
                DIAF_TRY(launch_classify_columns(n, nd, dtmp, kd, td, cc, dsorted, dmeta, nullptr, st));
                int32_t dh[ColumnClasses::kMax + 1] = {};
                DIAF_HIP_TRY(hipMemcpyAsync(dh, dmeta, sizeof(int32_t) * (ncls + 1),
                                            hipMemcpyDeviceToHost, st));
                DIAF_TRY(sync(st));
                std::vector<Seg> d;
                int off = 0;
                for (int c = 0; c < ncls; ++c) {
                    if (dh[c]) d.push_back({c, dsorted + off, dh[c]});
                    off += dh[c];
                }
                segs.insert(segs.begin(), d.begin(), d.end());
            }
            F->stats.count_deferred += nd;
        }
    }
    // Mid-size columns for unit-norm v (no Section 3.1 leverage rule, no
    // Section 3.2 constraint, |L_j| <= 8): the mid-size one-wave kernel takes
    // the classes it holds; the columns it hands back (more than 256 rows of
    // B_j with two or more entries, or |L_j| > 8) join the generic kernel's
    // list, sorted and classified again.
    const bool mid_ok = mode == DIAF_UNIT_V && ctx->opt_mid && !ctx->opt_generic_only &&
                        !spec->gram_fp32 && F->lmax <= 8 && !(spec->stab_r > 0.0) &&
                        fa.vrule != V_LEV_LOWER && fa.vrule != V_LEV_UPPER;
    if (mid_ok) {
        int nmid = 0;
        for (const Seg& g : segs)
            if (mid_supports<T>(cc.kcap[g.c], cc.tcap[g.c])) nmid += g.count;
        if (nmid > 0) {
            // the mid-size columns, gathered and sorted by the kernel's own
            // size classes (smaller LDS, higher occupancy, for |J_j| <= 32)
            std::vector<Seg> rest;
            int32_t *mdefl = nullptr, *mndef = nullptr, *mcols = nullptr, *msorted = nullptr;
            DIAF_TRY(scratch(&mdefl, nmid));
            DIAF_TRY(scratch(&mndef, 1));
            DIAF_TRY(scratch(&mcols, nmid));
            DIAF_TRY(scratch(&msorted, nmid));
            DIAF_TRY(clear_counter(mndef));
            int moff = 0;
            for (const Seg& g : segs) {
                if (!mid_supports<T>(cc.kcap[g.c], cc.tcap[g.c])) {
                    rest.push_back(g);
                    continue;
                }
                DIAF_HIP_TRY(hipMemcpyAsync(mcols + moff, g.cols, sizeof(int32_t) * g.count,
                                            hipMemcpyDeviceToDevice, st));
                moff += g.count;
            }
            ColumnClasses mcc{};
            mcc.ncls = mid_classes<T>(mcc.kcap, mcc.tcap);
            DIAF_TRY(launch_classify_columns(n, nmid, mcols, kd, td, mcc, msorted, dmeta, nullptr,
                                             st));
            int32_t mh[ColumnClasses::kMax + 1] = {};
            DIAF_HIP_TRY(hipMemcpyAsync(mh, dmeta, sizeof(int32_t) * (mcc.ncls + 1),
                                        hipMemcpyDeviceToHost, st));
            DIAF_TRY(sync(st));
            if (mh[mcc.ncls] != 0) return {DIAF_EINVAL, "internal: mid-size column classes"};
            int mo = 0;
            for (int c = 0; c < mcc.ncls; ++c) {
                if (mh[c] == 0) continue;
                fa.cols = msorted + mo;
                fa.ncols = mh[c];
                mo += mh[c];
                const int kcap = mcc.kcap[c], tcap = mcc.tcap[c];
                const FactorTune tune = ctx->ftune;
                DIAF_TRY(timed(-2, [fa, kcap, tcap, mdefl, mndef, tune](hipStream_t s) -> Err {
                    return launch_factor_mid<T>(fa, kcap, tcap, mdefl, mndef, tune, s);
                }));
                ++nb;
                F->stats.occ_mid = mid_occupancy<T>(kcap, tcap);
            }
            int32_t nd = 0;
            DIAF_TRY(read1(mndef, &nd, st));
            if (rec) rec->counters.push_back({mndef, nd});
            F->stats.cols_mid += nmid - nd;
            if (nd > 0) {
                int32_t *dtmp = nullptr, *dsorted = nullptr;
                DIAF_TRY(scratch(&dtmp, nd));
                DIAF_TRY(scratch(&dsorted, nd));
                DIAF_TRY(sort_columns(n, nd, mdefl, dtmp, st));
                DIAF_TRY(launch_classify_columns(n, nd, dtmp, kd, td, cc, dsorted, dmeta, nullptr, st));
                int32_t dh[ColumnClasses::kMax + 1] = {};
                DIAF_HIP_TRY(hipMemcpyAsync(dh, dmeta, sizeof(int32_t) * (ncls + 1),
                                            hipMemcpyDeviceToHost, st));
                DIAF_TRY(sync(st));
                std::vector<Seg> d;
                int off = 0;
                for (int c = 0; c < ncls; ++c) {
                    if (dh[c]) d.push_back({c, dsorted + off, dh[c]});
                    off += dh[c];
                }
                rest.insert(rest.begin(), d.begin(), d.end());
            }
            F->stats.count_deferred += nd;
            segs.swap(rest);
        }
    }
    for (const Seg& g : segs) {
        ++nb;
        fa.cols = g.cols;
        fa.ncols = g.count;
        const int kcap = cc.kcap[g.c], tcap = cc.tcap[g.c];
        int nslots = 1024;
        size_t gbytes = generic_global_bytes<T>(kcap, tcap, F->lmax, mode, nslots);
        void* gm = nullptr;
        if (gbytes) {
            DIAF_TRY(dmalloc((unsigned char**)&gm, gbytes));
            keep.push_back(gm);
        }
        const FactorTune tune = ctx->ftune;
        const int lcap = F->lmax;
        DIAF_TRY(timed(g.c, [fa, kcap, tcap, lcap, gm, nslots, tune](hipStream_t s) -> Err {
            return launch_factor_generic<T>(fa, kcap, tcap, lcap, gm, nslots, tune, s);
        }));
        F->stats.cols_generic_class[g.c] += g.count;
        F->stats.occ_generic_class[g.c] = generic_occupancy<T>(kcap, tcap, F->lmax, mode,
                                                               ctx->ftune);
    }
    DIAF_TRY(sync(st));
    double kms = 0;
    for (size_t q = 0; q < events.size(); ++q) {
        float ms = 0;
        DIAF_HIP_TRY(hipEventElapsedTime(&ms, events[q].first, events[q].second));
        kms += ms;
        if (ev_class[q] == -1) {
            F->stats.ms_small_kernel += ms;
            F->stats.launches_small += 1;
        } else if (ev_class[q] == -2) {
            F->stats.ms_mid_kernel += ms;
            F->stats.launches_mid += 1;
        } else {
            F->stats.ms_generic_class[ev_class[q]] += ms;
            F->stats.launches_generic_class[ev_class[q]] += 1;
        }
    }
    F->stats.ms_factor_kernels += kms;
    F->stats.factor_launches += (int32_t)events.size();
    if (nbuckets) *nbuckets = nb;
    return {};
}

template <class T>
Err assemble_v(diaf_ctx* ctx, diaf_factors* F)
{
    hipStream_t st = ctx->stream;
    const int n = (int)F->n;
    dfree(F->Vri);
    dfree(F->Vval);
    F->Vri = nullptr;
    F->Vval = nullptr;
    DIAF_TRY(exclusive_scan_i32(F->lcount, F->Vcp, n, st));
    int32_t nv = 0;
    DIAF_TRY(read1(F->Vcp + n, &nv, st));
    F->nnzV = nv;
    DIAF_TRY(dmalloc(&F->Vri, sizeof(int32_t) * (size_t)nv));
    DIAF_TRY(dmalloc(&F->Vval, sizeof(T) * (size_t)nv));
    DIAF_TRY(launch_compact_v<T>(n, F->lmax, F->lcount, F->Vcp, F->Vrows, (const T*)F->Vvals,
                                 F->Vri, (T*)F->Vval, st));
    return sync(st);
}

template <class T>
Err compute_stats(diaf_ctx* ctx, diaf_factors* F)
{
    hipStream_t st = ctx->stream;
    int32_t* counts = nullptr;
    double* nrm2 = nullptr;
    DIAF_TRY(dmalloc(&counts, sizeof(int32_t) * 8));
    DIAF_TRY(dmalloc(&nrm2, sizeof(double)));
    DIAF_HIP_TRY(hipMemsetAsync(counts, 0, sizeof(int32_t) * 8, st));
    DIAF_TRY(launch_flag_stats<T>((int)F->n, F->flags, F->r, counts, nrm2, st));
    int32_t c[8];
    double s = 0;
    DIAF_HIP_TRY(hipMemcpyAsync(c, counts, sizeof(c), hipMemcpyDeviceToHost, st));
    DIAF_HIP_TRY(hipMemcpyAsync(&s, nrm2, sizeof(double), hipMemcpyDeviceToHost, st));
    DIAF_TRY(sync(st));
    dfree(counts);
    dfree(nrm2);
    F->stats.count_rank_deficient = c[0];
    F->stats.count_gap_degenerate = c[1];
    F->stats.count_small_diag = c[2];
    F->stats.count_fell_back = c[3];
    F->stats.count_tie_edge = c[4];
    F->stats.count_stabilized = c[5];
    F->stats.count_no_diag = c[6];
    F->stats.count_null_choice = c[7];
    F->stats.nrm = sqrt(s);
    F->stats.n = F->n;
    F->stats.nnz_w = F->nnzW;
    F->stats.nnz_v = F->nnzV;
    return {};
}

Err pattern_hash(const diaf_csc* A, uint64_t* h, hipStream_t st)
{
    unsigned long long* d = nullptr;
    DIAF_TRY(dmalloc(&d, sizeof(unsigned long long)));
    Err e = launch_pattern_hash((int)A->n, A->nnz, A->colptr, A->rowidx, d, st);
    unsigned long long v = 0;
    if (e.code == DIAF_OK) e = read1(d, &v, st);
    dfree(d);
    *h = v;
    return e;
}

template <class T>
Err ensure_apply(diaf_ctx* ctx, diaf_factors* F)
{
    if (F->apply_ready) return {};
    hipStream_t st = ctx->stream;
    const int n = (int)F->n;
    if (F->vtri == 2) return {DIAF_EUNSUPPORTED, "apply: V is neither triangular nor diagonal"};
    DIAF_TRY(dmalloc(&F->Wrp, sizeof(int32_t) * (n + 1)));
    DIAF_TRY(dmalloc(&F->Wci, sizeof(int32_t) * (size_t)F->nnzW));
    DIAF_TRY(dmalloc(&F->Wcv, sizeof(T) * (size_t)F->nnzW));
    DIAF_TRY(csc_to_csr<T>(n, F->nnzW, F->Jcp, F->Jri, (const T*)F->Wval, F->Wrp, F->Wci,
                           (T*)F->Wcv, st));
    if (F->vtri == 3) {
        // block diagonal V: LU with partial pivoting of every block
        DIAF_TRY(dmalloc(&F->tmp, sizeof(T) * n));
        DIAF_TRY(dmalloc(&F->blu, sizeof(T) * (size_t)F->lu_elems));
        DIAF_TRY(dmalloc(&F->bperm, sizeof(int32_t) * n));
        int32_t* bad = nullptr;
        DIAF_TRY(dmalloc(&bad, sizeof(int32_t)));
        DIAF_HIP_TRY(hipMemsetAsync(bad, 0, sizeof(int32_t), st));
        Err e = launch_block_lu<T>(F->nblk, F->bstart, F->boff, F->Vcp, F->Vri, (const T*)F->Vval,
                                   (T*)F->blu, F->bperm, bad, st);
        int32_t nb = 0;
        if (e.code == DIAF_OK) e = read1(bad, &nb, st);
        dfree(bad);
        DIAF_TRY(e);
        if (nb & (1 << 30)) return {DIAF_EDEVICE, "block diagonal V has an entry outside its block"};
        F->stats.count_zero_pivot = nb;
        F->stats.v_levels = 1;
        F->apply_ready = true;
        return {};
    }
    DIAF_TRY(dmalloc(&F->Vrp, sizeof(int32_t) * (n + 1)));
    DIAF_TRY(dmalloc(&F->Vci, sizeof(int32_t) * (size_t)F->nnzV));
    DIAF_TRY(dmalloc(&F->Vcv, sizeof(T) * (size_t)F->nnzV));
    DIAF_TRY(csc_to_csr<T>(n, F->nnzV, F->Vcp, F->Vri, (const T*)F->Vval, F->Vrp, F->Vci,
                           (T*)F->Vcv, st));
    DIAF_TRY(dmalloc(&F->tmp, sizeof(T) * n));
    DIAF_TRY(dmalloc(&F->ctl, sizeof(TrsvCtl)));
    DIAF_HIP_TRY(hipMemsetAsync(F->ctl, 0, sizeof(TrsvCtl), st));
    {
        int32_t* bad = nullptr;
        DIAF_TRY(dmalloc(&bad, sizeof(int32_t)));
        DIAF_HIP_TRY(hipMemsetAsync(bad, 0, sizeof(int32_t), st));
        DIAF_TRY(launch_diag_check<T>(n, F->Vrp, F->Vci, (const T*)F->Vcv, bad, st));
        int32_t nb = 0;
        DIAF_TRY(read1(bad, &nb, st));
        dfree(bad);
        F->stats.count_zero_pivot = nb;
    }
    DIAF_TRY(sync(st));
    F->apply_ready = true;
    if (F->stats.count_zero_pivot) return {};
    // the dependency depth of a triangular V is a diagnostic, taken on
    // request (diaf_factors_levels)
    F->stats.v_levels = (F->vtri == 1 || F->vtri == -1) ? 0 : 1;
    return {};
}

// Depth of the triangular dependency DAG of V (a sync-free level walk on the
// CSR copy), kept in the statistics.
template <class T>
Err compute_levels(diaf_ctx* ctx, diaf_factors* F)
{
    DIAF_TRY(ensure_apply<T>(ctx, F));
    if (!(F->vtri == 1 || F->vtri == -1)) {
        F->stats.v_levels = 1;  // diagonal or block diagonal: one step
        return {};
    }
    if (F->stats.v_levels > 0) return {};
    hipStream_t st = ctx->stream;
    const int n = (int)F->n;
    int32_t *lvl = nullptr, *mx = nullptr;
    struct FreeL {
        int32_t** a; int32_t** b;
        ~FreeL() { dfree(*a); dfree(*b); }
    } freel{&lvl, &mx};
    DIAF_TRY(dmalloc(&lvl, sizeof(int32_t) * n));
    DIAF_TRY(dmalloc(&mx, sizeof(int32_t)));
    DIAF_HIP_TRY(hipMemsetAsync(mx, 0, sizeof(int32_t), st));
    DIAF_TRY(launch_trsv_levels(n, F->Vrp, F->Vci, F->vtri > 0, lvl, F->ctl, mx, st));
    int32_t depth = 0;
    DIAF_TRY(read1(mx, &depth, st));
    TrsvCtl c{};
    DIAF_TRY(read1(F->ctl, &c, st));
    if (c.error) return {DIAF_EDEVICE, "triangular dependency walk exceeded its wait budget"};
    F->stats.v_levels = depth;
    return {};
}

// Right: t = V^{-1} x ; y = W t.  Left: t = W x ; y = V^{-1} t.  All on
// stream st, no host sync.  t (n entries) and ctl (the triangular solve's
// control words) are the factors' own buffers, or the caller's; prefilled:
// the triangular solve's output already holds its not-ready sentinel.
template <class T>
Err enqueue_apply_with(diaf_ctx* ctx, diaf_factors* F, const T* x, T* y, const int32_t* done,
                       hipStream_t st, T* t, TrsvCtl* ctl, bool prefilled = false)
{
    const int n = (int)F->n;
    const T* vin = x;
    T* vout = t;
    if (F->left) {
        DIAF_TRY(launch_spmv_csr<T>(n, F->nnzW, F->Wrp, F->Wci, (const T*)F->Wcv, x, t, done, st));
        vin = t;
        vout = y;
    }
    if (F->vtri == 0)
        DIAF_TRY(launch_diag_solve<T>(n, F->Vrp, F->Vci, (const T*)F->Vcv, vin, vout, done, st));
    else if (F->vtri == 3)
        DIAF_TRY(launch_block_solve<T>(F->nblk, F->bstart, F->boff, (const T*)F->blu, F->bperm, vin,
                                       vout, done, st));
    else
        DIAF_TRY(launch_trsv<T>(n, F->Vrp, F->Vci, (const T*)F->Vcv, F->vtri > 0, vin, vout,
                                ctl, done, ctx->trsv, st, prefilled));
    if (F->left) return {};
    return launch_spmv_csr<T>(n, F->nnzW, F->Wrp, F->Wci, (const T*)F->Wcv, (const T*)t, y, done,
                              st);
}

template <class T>
Err enqueue_apply(diaf_ctx* ctx, diaf_factors* F, const T* x, T* y, const int32_t* done,
                  hipStream_t st)
{
    return enqueue_apply_with<T>(ctx, F, x, y, done, st, (T*)F->tmp, F->ctl);
}

// The allocation-free apply: the same kernels as diaf_apply, with t and the
// control words in the device's fixed scratch array (cleared by a kernel),
// then a read of the control words' error flag.
template <class T>
Err apply_noalloc(diaf_ctx* ctx, diaf_factors* F, const T* x, T* y)
{
    const int n = (int)F->n;
    if ((size_t)n * sizeof(T) > NOALLOC_SCRATCH_BYTES - NOALLOC_CTL_BYTES)
        return {DIAF_EINVAL, "diaf_apply_noalloc: n = " + std::to_string(n) + " needs " +
                                 std::to_string((size_t)n * sizeof(T)) +
                                 " bytes of scratch; the limit is " +
                                 std::to_string(NOALLOC_SCRATCH_BYTES - NOALLOC_CTL_BYTES)};
    void* base = nullptr;
    DIAF_TRY(noalloc_scratch(ctx->device, &base));
    TrsvCtl* ctl = (TrsvCtl*)base;
    T* t = (T*)((unsigned char*)base + NOALLOC_CTL_BYTES);
    hipStream_t st = ctx->stream;
    DIAF_TRY(noalloc_clear(ctl, sizeof(TrsvCtl), st));
    DIAF_TRY(enqueue_apply_with<T>(ctx, F, x, y, nullptr, st, t, ctl));
    if (F->vtri == 1 || F->vtri == -1) {
        TrsvCtl c{};
        DIAF_HIP_TRY(hipMemcpyAsync(&c, ctl, sizeof(TrsvCtl), hipMemcpyDeviceToHost, st));
        DIAF_HIP_TRY(hipStreamSynchronize(st));
        if (c.error) return {DIAF_EDEVICE, "triangular solve exceeded its wait budget"};
    }
    return {};
}

template <class T>
Err factor_impl(diaf_ctx* ctx, const diaf_csc* A, const diaf_spec* spec, int mode,
                diaf_factors** out);
template <class T>
Err factor_left(diaf_ctx* ctx, const diaf_csc* A, const diaf_spec* spec, int mode,
                diaf_factors** out);
template <class T>
Err refactor_impl(diaf_ctx* ctx, const diaf_csc* A, diaf_factors* F);

}  // namespace

// ===========================================================================
// Exported functions
// ===========================================================================
extern "C" {

diaf_status diaf_ctx_create(diaf_ctx** ctx, int device, void* hip_stream)
{
    if (!ctx) return DIAF_EINVAL;
    *ctx = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) return DIAF_EDEVICE;
    if (device < 0 || device >= ndev) return DIAF_EINVAL;
    if (hipSetDevice(device) != hipSuccess) return DIAF_EDEVICE;
    // the allocation-free apply's scratch array: its address on this device
    if (diaf::noalloc_init(device).code != DIAF_OK) return DIAF_EDEVICE;
    auto* c = new diaf_ctx;
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    *ctx = c;
    return DIAF_OK;
}

void diaf_ctx_destroy(diaf_ctx* ctx)
{
    if (!ctx) return;
    if (hipSetDevice(ctx->device) == hipSuccess) {
        (void)hipDeviceSynchronize();
        release_kept(ctx->device);
    }
    if (ctx->gstream) (void)hipStreamDestroy(ctx->gstream);
    delete ctx;
}

const char* diaf_last_error(const diaf_ctx* ctx) { return ctx ? ctx->err.c_str() : ""; }

diaf_status diaf_ctx_get_option(const diaf_ctx* ctx, const char* key, int64_t* value)
{
    if (!ctx || !key || !value) return DIAF_EINVAL;
    std::string k(key);
    if (k == "generic_only") *value = ctx->opt_generic_only;
    else if (k == "mid") *value = ctx->opt_mid;
    else if (k == "solve_batch") *value = ctx->opt_batch;
    else if (k == "trsv_backoff") *value = ctx->trsv.backoff;
    else if (k == "trsv_waves") *value = ctx->trsv.waves;
    else if (k == "gate_small_diag") *value = ctx->opt_gate_small_diag;
    else if (k == "graph") *value = ctx->opt_graph;
    else if (k == "small_grid") *value = ctx->ftune.small_grid;
    else if (k == "generic_nt") *value = ctx->ftune.generic_nt;
    else if (k == "class_table") *value = ctx->opt_class_table;
    else if (k == "factor_graph") *value = ctx->opt_factor_graph;
    else return DIAF_EINVAL;
    return DIAF_OK;
}

diaf_status diaf_ctx_set_option(diaf_ctx* ctx, const char* key, int64_t value)
{
    if (!ctx || !key) return DIAF_EINVAL;
    std::string k(key);
    if (k == "generic_only") ctx->opt_generic_only = value;
    else if (k == "mid") ctx->opt_mid = value ? 1 : 0;
    else if (k == "solve_batch") ctx->opt_batch = value < 1 ? 1 : value;
    else if (k == "trsv_backoff") {
        if (value < 0 || value > 256)
            return fail(ctx, DIAF_EINVAL, "trsv_backoff must be in 0..256");
        ctx->trsv.backoff = (int)value;
    }
    else if (k == "gate_small_diag") ctx->opt_gate_small_diag = value ? 1 : 0;
    else if (k == "graph") ctx->opt_graph = value ? 1 : 0;
    else if (k == "small_grid") ctx->ftune.small_grid = value < 0 ? 0 : (int)value;
    else if (k == "generic_nt") {
        if (value != 0 && value != 64 && value != 128 && value != 256 && value != 512)
            return fail(ctx, DIAF_EINVAL, "generic_nt must be 0, 64, 128, 256 or 512");
        ctx->ftune.generic_nt = (int)value;
    }
    else if (k == "trsv_waves") {
        if (value != 1 && value != 2 && value != 4 && value != 8 && value != 16)
            return fail(ctx, DIAF_EINVAL, "trsv_waves must be 1, 2, 4, 8 or 16");
        ctx->trsv.waves = (int)value;
    }
    else if (k == "factor_graph") ctx->opt_factor_graph = value ? 1 : 0;
    else if (k == "class_table") {
        if (value < 0 || value >= kNumClassTables)
            return fail(ctx, DIAF_EINVAL,
                        "class_table must be in 0.." + std::to_string(kNumClassTables - 1));
        ctx->opt_class_table = value;
    }
    else return fail(ctx, DIAF_EINVAL, "unknown option " + k);
    return DIAF_OK;
}

diaf_status diaf_copy(diaf_ctx* ctx, void* dst, const void* src, size_t bytes)
{
    if (!ctx || (!dst && bytes) || (!src && bytes)) return DIAF_EINVAL;
    if (bytes == 0) return DIAF_OK;
    hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyDefault, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return fail(ctx, DIAF_EDEVICE, hipGetErrorString(e));
    return DIAF_OK;
}

diaf_status diaf_pattern_build(diaf_ctx* ctx, const diaf_csc* A, int32_t w_kind, int32_t w_topk,
                               int32_t* colptr_out, int32_t* rowidx_out, int64_t* nnz_host)
{
    if (!ctx) return DIAF_EINVAL;
    Err e = check_csc_host(A);
    if (e.code) return fail(ctx, e);
    if (!colptr_out || !nnz_host) return fail(ctx, DIAF_EINVAL, "NULL output");
    if (w_kind != DIAF_W_A && w_kind != DIAF_W_A2 && w_kind != DIAF_W_A_1HOP_TOPK &&
        w_kind != DIAF_W_ALG2_DIAG && w_kind != DIAF_W_ALG2_GS_UPPER &&
        w_kind != DIAF_W_ALG2_GS_LOWER)
        return fail(ctx, DIAF_EINVAL, "w_kind must be A, A2, A_1HOP_TOPK or ALG2_* (the "
                                      "sparsified powers: diaf_pattern_build_sparsified)");
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, DIAF_EDEVICE, "hipSetDevice");
    e = A->dtype == DIAF_F64 ? validate_A<double>(A, ctx->stream) : validate_A<zc>(A, ctx->stream);
    if (e.code) return fail(ctx, e);
    int32_t* none = nullptr;
    e = A->dtype == DIAF_F64
            ? build_pattern<double>(A, w_kind, w_topk, colptr_out, &none, nnz_host, false,
                                    rowidx_out, ctx->stream)
            : build_pattern<zc>(A, w_kind, w_topk, colptr_out, &none, nnz_host, false, rowidx_out,
                                ctx->stream);
    if (e.code) return fail(ctx, e);
    return DIAF_OK;
}

diaf_status diaf_pattern_build_sparsified(diaf_ctx* ctx, const diaf_csc* A,
                                          const diaf_sparsify* prm, int32_t* colptr_out,
                                          int32_t* rowidx_out, int64_t* nnz_host)
{
    if (!ctx) return DIAF_EINVAL;
    Err e = check_csc_host(A);
    if (e.code) return fail(ctx, e);
    if (!colptr_out || !nnz_host) return fail(ctx, DIAF_EINVAL, "NULL output");
    e = check_sparsify(prm);
    if (e.code) return fail(ctx, e);
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, DIAF_EDEVICE, "hipSetDevice");
    e = A->dtype == DIAF_F64 ? validate_A<double>(A, ctx->stream) : validate_A<zc>(A, ctx->stream);
    if (e.code) return fail(ctx, e);
    int32_t* none = nullptr;
    e = build_sparsified(A, prm, colptr_out, &none, nnz_host, false, rowidx_out, ctx->stream);
    if (e.code) return fail(ctx, e);
    return DIAF_OK;
}

diaf_status diaf_factor(diaf_ctx* ctx, const diaf_csc* A, const diaf_spec* spec, int32_t mode,
                        diaf_factors** out)
{
    if (!ctx) return DIAF_EINVAL;
    if (!out) return fail(ctx, DIAF_EINVAL, "out is NULL");
    *out = nullptr;
    Err e = check_csc_host(A);
    if (e.code) return fail(ctx, e);
    if (!spec) return fail(ctx, DIAF_EINVAL, "spec is NULL");
    if (mode != DIAF_UNIT_V && mode != DIAF_UNIT_W) return fail(ctx, DIAF_EINVAL, "bad norm mode");
    e = check_spec(A, spec, mode);
    if (e.code) return fail(ctx, e);
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, DIAF_EDEVICE, "hipSetDevice");
    if (spec->left)
        e = A->dtype == DIAF_F64 ? factor_left<double>(ctx, A, spec, mode, out)
                                 : factor_left<zc>(ctx, A, spec, mode, out);
    else
        e = A->dtype == DIAF_F64 ? factor_impl<double>(ctx, A, spec, mode, out)
                                 : factor_impl<zc>(ctx, A, spec, mode, out);
    if (e.code) return fail(ctx, e);
    return DIAF_OK;
}

diaf_status diaf_refactor(diaf_ctx* ctx, const diaf_csc* A, diaf_factors* F)
{
    if (!ctx) return DIAF_EINVAL;
    if (!F) return fail(ctx, DIAF_EINVAL, "factors are NULL");
    Err e = check_csc_host(A);
    if (e.code) return fail(ctx, e);
    if (F->ctx != ctx) return fail(ctx, DIAF_EINVAL, "refactor: factors of another context");
    if (F->left) return fail(ctx, DIAF_EUNSUPPORTED, "refactor: not for the left variant");
    const int wk = F->spec.w_kind;
    if (!(wk == DIAF_W_A || wk == DIAF_W_A2 || wk == DIAF_W_EXPLICIT || wk == DIAF_W_ALG2_DIAG ||
          wk == DIAF_W_ALG2_GS_UPPER || wk == DIAF_W_ALG2_GS_LOWER))
        return fail(ctx, DIAF_EUNSUPPORTED,
                    "refactor: the W pattern depends on the values (1-hop, sparsified powers, "
                    "learned); factor afresh");
    if (A->n != F->n || A->nnz != F->src_nnz || A->dtype != F->dtype || A->colptr != F->src_cp ||
        A->rowidx != F->src_ri || A->val != F->src_val)
        return fail(ctx, DIAF_EINVAL, "refactor: A must be the matrix the factors were built "
                                      "from (same buffers), with new values in place");
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, DIAF_EDEVICE, "hipSetDevice");
    e = A->dtype == DIAF_F64 ? refactor_impl<double>(ctx, A, F) : refactor_impl<zc>(ctx, A, F);
    if (e.code) return fail(ctx, e);
    return DIAF_OK;
}

diaf_status diaf_factors_view(const diaf_factors* F, diaf_view* v)
{
    if (!F || !v) return DIAF_EINVAL;
    v->n = F->n;
    v->nnz_w = F->nnzW;
    v->nnz_v = F->nnzV;
    v->dtype = F->dtype;
    v->vtri = F->vtri;
    v->Wcp = F->Jcp;
    v->Wri = F->Jri;
    v->Wval = F->Wval;
    v->Vcp = F->Vcp;
    v->Vri = F->Vri;
    v->Vval = F->Vval;
    v->r = F->r;
    v->flags = F->flags;
    v->lcount = F->lcount;
    return DIAF_OK;
}

diaf_status diaf_factors_stats(const diaf_factors* F, diaf_stats* s)
{
    if (!F || !s) return DIAF_EINVAL;
    *s = F->stats;
    return DIAF_OK;
}

diaf_status diaf_factors_levels(diaf_ctx* ctx, const diaf_factors* Fc, int32_t* levels)
{
    if (!ctx) return DIAF_EINVAL;
    if (!Fc || !levels) return fail(ctx, DIAF_EINVAL, "NULL argument");
    auto* F = const_cast<diaf_factors*>(Fc);
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, DIAF_EDEVICE, "hipSetDevice");
    Err e = F->dtype == DIAF_F64 ? compute_levels<double>(ctx, F) : compute_levels<zc>(ctx, F);
    if (e.code) return fail(ctx, e);
    *levels = F->stats.v_levels;
    return DIAF_OK;
}

void diaf_factors_destroy(diaf_factors* F) { free_factors(F); }

diaf_status diaf_apply_noalloc(diaf_ctx* ctx, const diaf_factors* Fc, const void* x, void* y)
{
    if (!ctx) return DIAF_EINVAL;
    if (!Fc || !x || !y) return fail(ctx, DIAF_EINVAL, "NULL argument");
    auto* F = const_cast<diaf_factors*>(Fc);
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, DIAF_EDEVICE, "hipSetDevice");
    if (!F->apply_ready)
        return fail(ctx, DIAF_EINVAL,
                    "diaf_apply_noalloc: the factors are not prepared for applying (their "
                    "row-oriented copies are built by the first diaf_apply or diaf_solve)");
    if (F->stats.count_zero_pivot)
        return fail(ctx, DIAF_ESINGULAR, std::to_string(F->stats.count_zero_pivot) +
                                             " zero or non-finite pivots in V");
    Err e = F->dtype == DIAF_F64
                ? apply_noalloc<double>(ctx, F, (const double*)x, (double*)y)
                : apply_noalloc<zc>(ctx, F, (const zc*)x, (zc*)y);
    if (e.code) return fail(ctx, e);
    return DIAF_OK;
}

diaf_status diaf_apply(diaf_ctx* ctx, const diaf_factors* Fc, const void* x, void* y)
{
    if (!ctx) return DIAF_EINVAL;
    if (!Fc || !x || !y) return fail(ctx, DIAF_EINVAL, "NULL argument");
    auto* F = const_cast<diaf_factors*>(Fc);
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, DIAF_EDEVICE, "hipSetDevice");
    Err e;
    e = F->dtype == DIAF_F64 ? ensure_apply<double>(ctx, F) : ensure_apply<zc>(ctx, F);
    if (e.code) return fail(ctx, e);
    if (F->stats.count_zero_pivot)
        return fail(ctx, DIAF_ESINGULAR, std::to_string(F->stats.count_zero_pivot) +
                                             " zero or non-finite pivots in V");
    if (F->dtype == DIAF_F64)
        e = enqueue_apply<double>(ctx, F, (const double*)x, (double*)y, nullptr, ctx->stream);
    else
        e = enqueue_apply<zc>(ctx, F, (const zc*)x, (zc*)y, nullptr, ctx->stream);
    if (e.code) return fail(ctx, e);
    if (F->stats.count_zero_pivot)
        return fail(ctx, DIAF_ESINGULAR, std::to_string(F->stats.count_zero_pivot) +
                                             " zero or non-finite pivots in V");
    if (F->vtri == 1 || F->vtri == -1) {
        TrsvCtl c{};
        e = read1(F->ctl, &c, ctx->stream);
        if (e.code) return fail(ctx, e);
        if (c.error) return fail(ctx, DIAF_EDEVICE, "triangular solve exceeded its wait budget");
    }
    return DIAF_OK;
}

}  // extern "C"

// ===========================================================================
// Factor and solve implementations
// ===========================================================================
namespace {

// Learned proposal: C = pattern(A^2), features, MLP scores, J = {j} U {i : score >= 0}.
template <class T>
Err learned_pattern(diaf_ctx* ctx, const diaf_csc* A, const diaf_model* M, diaf_factors* F,
                    int32_t** Ccp, int32_t** Cri, int64_t* nnzC)
{
    hipStream_t st = ctx->stream;
    const int n = (int)A->n;
    DIAF_TRY(dmalloc(Ccp, sizeof(int32_t) * (n + 1)));
    DIAF_TRY(build_pattern<T>(A, DIAF_W_A2, 0, *Ccp, Cri, nnzC, true, nullptr, st));
    float *feat = nullptr, *scores = nullptr;
    DIAF_TRY(dmalloc(&feat, sizeof(float) * 16 * (size_t)*nnzC));
    DIAF_TRY(dmalloc(&scores, sizeof(float) * (size_t)*nnzC));
    DIAF_TRY(launch_features<T>(n, A->colptr, A->rowidx, (const T*)A->val, *Ccp, *Cri, feat, st));
    DIAF_TRY(launch_mlp_forward(M->params, feat, *nnzC, scores, st));
    int32_t* cnt = nullptr;
    DIAF_TRY(dmalloc(&cnt, sizeof(int32_t) * (n + 1)));
    DIAF_TRY(launch_pattern_from_scores(n, *Ccp, *Cri, scores, cnt, nullptr, nullptr, st));
    DIAF_TRY(exclusive_scan_i32(cnt, F->Jcp, n, st));
    int32_t tot = 0;
    DIAF_TRY(read1(F->Jcp + n, &tot, st));
    F->nnzW = tot;
    DIAF_TRY(dmalloc(&F->Jri, sizeof(int32_t) * (size_t)tot));
    DIAF_TRY(launch_pattern_from_scores(n, *Ccp, *Cri, scores, nullptr, F->Jcp, F->Jri, st));
    DIAF_TRY(sync(st));
    dfree(feat);
    dfree(scores);
    dfree(cnt);
    return {};
}

// Residual gate: a column whose normalised residual r_j / s_j exceeds
// gate_tau (s_j = 1 for unit-norm v, ||A(:,J_j)||_F for unit-norm w) is
// refactored with the candidate pattern C_j = pattern(A^2)(:, j).
template <class T>
Err gate_and_fallback(diaf_ctx* ctx, const diaf_csc* A, const diaf_spec* spec, int mode,
                      diaf_factors* F, const int32_t* Ccp, const int32_t* Cri, int64_t nnzC)
{
    hipStream_t st = ctx->stream;
    const int n = (int)F->n;
    std::vector<double> r(n), bn(n), dom(n, INFINITY);
    std::vector<uint32_t> fl0(n);
    DIAF_HIP_TRY(hipMemcpyAsync(r.data(), F->r, sizeof(double) * n, hipMemcpyDeviceToHost, st));
    DIAF_HIP_TRY(hipMemcpyAsync(bn.data(), F->bnorm, sizeof(double) * n, hipMemcpyDeviceToHost, st));
    DIAF_HIP_TRY(hipMemcpyAsync(fl0.data(), F->flags, sizeof(uint32_t) * n, hipMemcpyDeviceToHost,
                                st));
    DevBlocks blocks;  // freed on every return path
    if (spec->gate_dom > 0.0) {
        double* domd = nullptr;
        DIAF_TRY(dmalloc(&domd, sizeof(double) * n));
        blocks.keep(domd);
        DIAF_TRY(launch_col_dominance<T>(n, F->lmax, F->Vrows, (const T*)F->Vvals, F->lcount,
                                         domd, st));
        DIAF_HIP_TRY(hipMemcpyAsync(dom.data(), domd, sizeof(double) * n, hipMemcpyDeviceToHost,
                                    st));
        DIAF_TRY(sync(st));
    }
    DIAF_TRY(sync(st));
    std::vector<uint8_t> fb(n, 0);
    std::vector<int32_t> list;
    // a proposal is rejected when its normalised residual exceeds the gate,
    // when its V column is not diagonally dominant enough (chains of such
    // columns make the triangular solve with V grow exponentially) or, unless
    // switched off, when V's diagonal entry is negligible (Section 3.2)
    const uint32_t reject = ctx->opt_gate_small_diag ? DIAF_FLAG_SMALL_DIAG : 0u;
    for (int j = 0; j < n; ++j) {
        double sj = mode == DIAF_UNIT_V ? 1.0 : bn[j];
        double q = sj > 0 ? r[j] / sj : r[j];
        if (!(q <= spec->gate_tau) || (fl0[j] & reject) || !(dom[j] >= spec->gate_dom)) {
            fb[j] = 1;
            list.push_back(j);
        }
    }
    if (list.empty()) return {};
    uint8_t* fbd = nullptr;
    int32_t *cnt = nullptr, *Jcp2 = nullptr, *Jri2 = nullptr;
    T* W2 = nullptr;
    DIAF_TRY(dmalloc(&fbd, n));
    blocks.keep(fbd);
    DIAF_TRY(dmalloc(&cnt, sizeof(int32_t) * (n + 1)));
    blocks.keep(cnt);
    DIAF_TRY(dmalloc(&Jcp2, sizeof(int32_t) * (n + 1)));
    blocks.keep(Jcp2);
    DIAF_HIP_TRY(hipMemcpyAsync(fbd, fb.data(), n, hipMemcpyHostToDevice, st));
    DIAF_TRY(launch_fallback_count(n, F->Jcp, Ccp, fbd, cnt, st));
    DIAF_TRY(exclusive_scan_i32(cnt, Jcp2, n, st));
    int32_t tot = 0;
    DIAF_TRY(read1(Jcp2 + n, &tot, st));
    DIAF_TRY(dmalloc(&Jri2, sizeof(int32_t) * (size_t)tot));
    blocks.keep(Jri2);
    DIAF_TRY(dmalloc(&W2, sizeof(T) * (size_t)tot));
    blocks.keep(W2);
    DIAF_TRY(launch_fallback_fill<T>(n, F->Jcp, F->Jri, (const T*)F->Wval, Ccp, Cri, fbd, Jcp2,
                                     Jri2, W2, F->flags, st));
    DIAF_TRY(sync(st));
    dfree(F->Jcp); dfree(F->Jri); dfree(F->Wval);
    F->Jcp = Jcp2; F->Jri = Jri2; F->Wval = W2; F->nnzW = tot;
    blocks.release(Jcp2);  // now owned by the factors
    blocks.release(Jri2);
    blocks.release(W2);
    DIAF_TRY(factor_columns<T>(ctx, A, spec, mode, F, &list, nullptr));
    // the refactor rewrote the flags of these columns: mark them again
    std::vector<uint32_t> fl(n);
    DIAF_HIP_TRY(hipMemcpyAsync(fl.data(), F->flags, sizeof(uint32_t) * n, hipMemcpyDeviceToHost, st));
    DIAF_TRY(sync(st));
    for (int32_t j : list) fl[j] |= DIAF_FLAG_FELL_BACK;
    DIAF_HIP_TRY(hipMemcpyAsync(F->flags, fl.data(), sizeof(uint32_t) * n, hipMemcpyHostToDevice, st));
    DIAF_TRY(sync(st));
    (void)nnzC;
    return {};
}

template <class T>
Err factor_impl(diaf_ctx* ctx, const diaf_csc* A, const diaf_spec* spec, int mode,
                diaf_factors** out)
{
    hipStream_t st = ctx->stream;
    const int n = (int)A->n;
    DIAF_TRY(validate_A<T>(A, st));
    std::unique_ptr<diaf_factors, void (*)(diaf_factors*)> F(new diaf_factors, free_factors);
    int32_t *Ccp = nullptr, *Cri = nullptr;  // learned path: candidate pattern pattern(A^2)
    int64_t nnzC = 0;
    struct CFree {
        int32_t** a; int32_t** b;
        ~CFree() { dfree(*a); dfree(*b); }
    } cfree{&Ccp, &Cri};
    F->ctx = ctx;
    F->n = n;
    F->dtype = A->dtype;
    F->mode = mode;
    F->vtri = vtri_of(spec->v_kind);
    hipEvent_t ev[4];
    for (auto& e : ev) DIAF_HIP_TRY(hipEventCreate(&e));
    DIAF_HIP_TRY(hipEventRecord(ev[0], st));
    // ---- W pattern ----
    DIAF_TRY(dmalloc(&F->Jcp, sizeof(int32_t) * (n + 1)));
    if (spec->w_kind == DIAF_W_EXPLICIT) {
        DIAF_TRY(validate_pattern(spec->w_explicit, n, 1, "W pattern", st));
        F->nnzW = spec->w_explicit->nnz;
        DIAF_TRY(dmalloc(&F->Jri, sizeof(int32_t) * (size_t)F->nnzW));
        DIAF_HIP_TRY(hipMemcpyAsync(F->Jcp, spec->w_explicit->colptr, sizeof(int32_t) * (n + 1),
                                    hipMemcpyDeviceToDevice, st));
        DIAF_HIP_TRY(hipMemcpyAsync(F->Jri, spec->w_explicit->rowidx,
                                    sizeof(int32_t) * (size_t)F->nnzW, hipMemcpyDeviceToDevice, st));
    } else if (spec->w_kind == DIAF_W_LEARNED) {
        if (!spec->model) return {DIAF_EINVAL, "learned W pattern: model is NULL"};
        DIAF_TRY(learned_pattern<T>(ctx, A, spec->model, F.get(), &Ccp, &Cri, &nnzC));
    } else {
        DIAF_TRY(build_pattern<T>(A, spec->w_kind, spec->w_topk, F->Jcp, &F->Jri, &F->nnzW, true,
                                  nullptr, st, &spec->sparsify));
    }
    DIAF_HIP_TRY(hipEventRecord(ev[1], st));
    // ---- V pattern capacity ----
    int lmax = 1;
    if (spec->v_kind == DIAF_V_TOPK_LOWER || spec->v_kind == DIAF_V_TOPK_UPPER ||
        spec->v_kind == DIAF_V_LEV_LOWER || spec->v_kind == DIAF_V_LEV_UPPER) {
        lmax = spec->v_count;
    } else if (spec->v_kind == DIAF_V_GS_LOWER || spec->v_kind == DIAF_V_GS_UPPER) {
        std::vector<int32_t> cp(n + 1);
        DIAF_HIP_TRY(hipMemcpyAsync(cp.data(), A->colptr, sizeof(int32_t) * (n + 1),
                                    hipMemcpyDeviceToHost, st));
        DIAF_TRY(sync(st));
        for (int j = 0; j < n; ++j) lmax = std::max(lmax, cp[j + 1] - cp[j]);
    } else if (spec->v_kind == DIAF_V_EXPLICIT) {
        DIAF_TRY(validate_pattern(spec->v_explicit, n, 0, "V pattern", st));
        std::vector<int32_t> cp(n + 1), ri(spec->v_explicit->nnz);
        DIAF_HIP_TRY(hipMemcpyAsync(cp.data(), spec->v_explicit->colptr, sizeof(int32_t) * (n + 1),
                                    hipMemcpyDeviceToHost, st));
        DIAF_HIP_TRY(hipMemcpyAsync(ri.data(), spec->v_explicit->rowidx,
                                    sizeof(int32_t) * ri.size(), hipMemcpyDeviceToHost, st));
        DIAF_TRY(sync(st));
        bool up = true, lo = true, dg = true;
        for (int j = 0; j < n; ++j) {
            lmax = std::max(lmax, cp[j + 1] - cp[j]);
            for (int p = cp[j]; p < cp[j + 1]; ++p) {
                up &= ri[p] <= j;
                lo &= ri[p] >= j;
                dg &= ri[p] == j;
            }
        }
        F->vtri = dg ? 0 : (up ? 1 : (lo ? -1 : 2));
    } else if (spec->v_kind == DIAF_V_BLOCK || spec->v_kind == DIAF_V_TOPK_BLOCK) {
        DIAF_TRY(setup_blocks(spec, n, F.get(), st));
        if (spec->v_kind == DIAF_V_TOPK_BLOCK) {
            lmax = spec->v_count;
        } else {
            // the pattern of D: the rows of each column of A inside its block
            int32_t* cnt = nullptr;
            DIAF_TRY(dmalloc(&cnt, sizeof(int32_t) * (n + 1)));
            Err e = launch_block_vpattern(n, A->colptr, A->rowidx, F->vblk, cnt, nullptr, nullptr,
                                          st);
            std::vector<int32_t> ch(n);
            if (e.code == DIAF_OK) e = dmalloc(&F->vpat_cp, sizeof(int32_t) * (n + 1));
            if (e.code == DIAF_OK) e = exclusive_scan_i32(cnt, F->vpat_cp, n, st);
            if (e.code == DIAF_OK && hipMemcpyAsync(ch.data(), cnt, sizeof(int32_t) * n,
                                                    hipMemcpyDeviceToHost, st) != hipSuccess)
                e = {DIAF_EDEVICE, "copy of the block V counts"};
            int32_t tot = 0;
            if (e.code == DIAF_OK) e = read1(F->vpat_cp + n, &tot, st);
            dfree(cnt);
            DIAF_TRY(e);
            for (int j = 0; j < n; ++j) lmax = std::max(lmax, ch[j]);
            DIAF_TRY(dmalloc(&F->vpat_ri, sizeof(int32_t) * (size_t)(tot > 0 ? tot : 1)));
            DIAF_TRY(launch_block_vpattern(n, A->colptr, A->rowidx, F->vblk, nullptr, F->vpat_cp,
                                           F->vpat_ri, st));
        }
    }
    if (lmax > 256) return {DIAF_EUNSUPPORTED, "V pattern with more than 256 rows in a column"};
    F->lmax = lmax;
    // ---- outputs ----
    DIAF_TRY(dmalloc(&F->Wval, sizeof(T) * (size_t)F->nnzW));
    DIAF_TRY(dmalloc(&F->Vrows, sizeof(int32_t) * (size_t)n * lmax));
    DIAF_TRY(dmalloc(&F->Vvals, sizeof(T) * (size_t)n * lmax));
    DIAF_TRY(dmalloc(&F->Vcp, sizeof(int32_t) * (n + 1)));
    DIAF_TRY(dmalloc(&F->r, sizeof(double) * n));
    DIAF_TRY(dmalloc(&F->bnorm, sizeof(double) * n));
    DIAF_TRY(dmalloc(&F->flags, sizeof(uint32_t) * n));
    DIAF_TRY(dmalloc(&F->lcount, sizeof(int32_t) * n));
    int nb = 0;
    DIAF_TRY(factor_columns<T>(ctx, A, spec, mode, F.get(), nullptr, &nb));
    F->stats.nbuckets = nb;
    if (spec->w_kind == DIAF_W_LEARNED)
        DIAF_TRY(gate_and_fallback<T>(ctx, A, spec, mode, F.get(), Ccp, Cri, nnzC));
    DIAF_HIP_TRY(hipEventRecord(ev[2], st));
    DIAF_TRY(assemble_v<T>(ctx, F.get()));
    DIAF_HIP_TRY(hipEventRecord(ev[3], st));
    DIAF_TRY(compute_stats<T>(ctx, F.get()));
    float ms[3] = {0, 0, 0};
    for (int i = 0; i < 3; ++i) DIAF_HIP_TRY(hipEventElapsedTime(&ms[i], ev[i], ev[i + 1]));
    for (auto& e : ev) (void)hipEventDestroy(e);
    F->stats.ms_pattern = ms[0];
    F->stats.ms_factor = ms[1];
    F->stats.ms_assemble = ms[2];
    // what diaf_refactor needs: the spec, the matrix buffers, the pattern's
    // fingerprint
    F->spec = *spec;
    F->src_cp = A->colptr;
    F->src_ri = A->rowidx;
    F->src_val = A->val;
    F->src_nnz = A->nnz;
    DIAF_TRY(pattern_hash(A, &F->pat_hash, st));
    *out = F.release();
    return {};
}

// Refactor F in place for new values of the matrix it was built from (same
// buffers, same pattern): the W pattern and the V pattern capacity are
// kept; the factor kernels run again (the first time eagerly, recording
// their launches; for unit-norm v later calls replay them as one captured
// graph), then V is assembled and the statistics taken again.  The apply
// structures are rebuilt on the next apply.
template <class T>
Err refactor_impl(diaf_ctx* ctx, const diaf_csc* A, diaf_factors* F)
{
    hipStream_t st = ctx->stream;
    const int n = (int)A->n;
    DIAF_TRY(validate_A<T>(A, st));
    uint64_t h = 0;
    DIAF_TRY(pattern_hash(A, &h, st));
    if (h != F->pat_hash)
        return {DIAF_EINVAL, "refactor: the pattern of A differs from the one the factors were "
                             "built from"};
    // the apply structures of the old values
    for (void** p : {(void**)&F->Wrp, (void**)&F->Wci, (void**)&F->Vrp, (void**)&F->Vci,
                     &F->Wcv, &F->Vcv, &F->tmp, (void**)&F->ctl, &F->blu, (void**)&F->bperm}) {
        dfree(*p);
        *p = nullptr;
    }
    F->apply_ready = false;
    hipEvent_t ev[3];
    for (auto& e : ev) DIAF_HIP_TRY(hipEventCreate(&e));
    struct EvFree {
        hipEvent_t* e;
        ~EvFree() { for (int i = 0; i < 3; ++i) (void)hipEventDestroy(e[i]); }
    } evfree{ev};
    DIAF_HIP_TRY(hipEventRecord(ev[0], st));
    const bool graph = F->mode == DIAF_UNIT_V && ctx->opt_factor_graph;
    if (graph && F->plan && F->plan->exec) {
        DIAF_HIP_TRY(hipGraphLaunch(F->plan->exec, st));
        std::vector<int32_t> got(F->plan->counters.size());
        for (size_t q = 0; q < got.size(); ++q)
            DIAF_HIP_TRY(hipMemcpyAsync(&got[q], F->plan->counters[q].first, sizeof(int32_t),
                                        hipMemcpyDeviceToHost, st));
        DIAF_TRY(sync(st));
        for (size_t q = 0; q < got.size(); ++q)
            if (got[q] != F->plan->counters[q].second)
                return {DIAF_EINVAL, "refactor: the columns handed between the factor kernels "
                                     "changed; factor afresh"};
        const diaf_stats keep = F->stats;
        F->stats = F->plan->stats;
        F->stats.ms_pattern = keep.ms_pattern;
    } else {
        // eager pass (recording it when a graph will replay it)
        FactorPlan* rec = nullptr;
        if (graph) {
            if (F->plan) {
                if (F->plan->exec) (void)hipGraphExecDestroy(F->plan->exec);
                if (F->plan->graph) (void)hipGraphDestroy(F->plan->graph);
                for (void* p : F->plan->bufs) dfree(p);
                delete F->plan;
            }
            F->plan = new FactorPlan;
            rec = F->plan;
        }
        const double pattern_ms = F->stats.ms_pattern;
        std::memset(&F->stats, 0, sizeof(F->stats));
        F->stats.ms_pattern = pattern_ms;
        int nb = 0;
        DIAF_TRY(factor_columns<T>(ctx, A, &F->spec, F->mode, F, nullptr, &nb, rec));
        F->stats.nbuckets = nb;
        if (rec) {
            // captured on the library stream (the caller's may be the null
            // stream, which cannot be captured); replayed on the caller's
            rec->stats = F->stats;
            if (!ctx->gstream)
                DIAF_HIP_TRY(hipStreamCreateWithFlags(&ctx->gstream, hipStreamNonBlocking));
            hipStream_t cs = ctx->gstream;
            DIAF_HIP_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
            Err ce{};
            for (auto& L : rec->launches) {
                ce = L(cs);
                if (ce.code) break;
            }
            hipGraph_t g = nullptr;
            const hipError_t he = hipStreamEndCapture(cs, &g);
            DIAF_TRY(ce);
            if (he != hipSuccess || !g) return {DIAF_EDEVICE, "refactor: graph capture failed"};
            rec->graph = g;
            DIAF_HIP_TRY(hipGraphInstantiate(&rec->exec, g, nullptr, nullptr, 0));
        }
    }
    DIAF_HIP_TRY(hipEventRecord(ev[1], st));
    DIAF_TRY(assemble_v<T>(ctx, F));
    DIAF_HIP_TRY(hipEventRecord(ev[2], st));
    DIAF_TRY(compute_stats<T>(ctx, F));
    float ms[2] = {0, 0};
    for (int i = 0; i < 2; ++i) DIAF_HIP_TRY(hipEventElapsedTime(&ms[i], ev[i], ev[i + 1]));
    F->stats.ms_factor = ms[0];
    F->stats.ms_assemble = ms[1];
    if (graph && F->plan && F->plan->exec) F->stats.ms_factor_kernels = ms[0];
    (void)n;
    return {};
}

// In-place conjugate transpose of a CSC matrix held in F (new arrays; the
// CSR of X is the CSC of X^T).
template <class T>
Err conj_transpose_csc(int n, int64_t nnz, int32_t** cp, int32_t** ri, void** val, hipStream_t st)
{
    int32_t *rp = nullptr, *ci = nullptr;
    T* cv = nullptr;
    Err e = dmalloc(&rp, sizeof(int32_t) * (n + 1));
    if (e.code == DIAF_OK) e = dmalloc(&ci, sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
    if (e.code == DIAF_OK) e = dmalloc(&cv, sizeof(T) * (size_t)(nnz > 0 ? nnz : 1));
    if (e.code == DIAF_OK) e = csc_to_csr<T>(n, nnz, *cp, *ri, (const T*)*val, rp, ci, cv, st);
    if (e.code == DIAF_OK) e = launch_conj<T>(nnz, cv, st);
    if (e.code == DIAF_OK) e = sync(st);
    if (e.code != DIAF_OK) {
        dfree(rp); dfree(ci); dfree(cv);
        return e;
    }
    dfree(*cp); dfree(*ri); dfree(*val);
    *cp = rp;
    *ri = ci;
    *val = cv;
    return {};
}

// Left variant (the remarks of Section 4 on left and right approximate
// inverses): W A ~ V row by row is A^* W^* ~ V^* column by column, so the
// columnwise method runs on A^* and its factors are conjugate-transposed:
// W = W~^*, V = V~^* (the triangle of V flips), M = V^{-1} W.
template <class T>
Err factor_left(diaf_ctx* ctx, const diaf_csc* A, const diaf_spec* spec, int mode,
                diaf_factors** out)
{
    hipStream_t st = ctx->stream;
    const int n = (int)A->n;
    DIAF_TRY(validate_A<T>(A, st));
    int32_t *rp = nullptr, *ci = nullptr;
    T* cv = nullptr;
    struct Free3 {
        int32_t** a; int32_t** b; T** c;
        ~Free3() { dfree(*a); dfree(*b); dfree(*c); }
    } f3{&rp, &ci, &cv};
    DIAF_TRY(dmalloc(&rp, sizeof(int32_t) * (n + 1)));
    DIAF_TRY(dmalloc(&ci, sizeof(int32_t) * (size_t)A->nnz));
    DIAF_TRY(dmalloc(&cv, sizeof(T) * (size_t)A->nnz));
    DIAF_TRY(csc_to_csr<T>(n, A->nnz, A->colptr, A->rowidx, (const T*)A->val, rp, ci, cv, st));
    DIAF_TRY(launch_conj<T>(A->nnz, cv, st));
    diaf_csc Ah = *A;
    Ah.colptr = rp;
    Ah.rowidx = ci;
    Ah.val = cv;
    diaf_factors* F = nullptr;
    DIAF_TRY(factor_impl<T>(ctx, &Ah, spec, mode, &F));
    Err e = conj_transpose_csc<T>(n, F->nnzW, &F->Jcp, &F->Jri, &F->Wval, st);
    if (e.code == DIAF_OK) e = conj_transpose_csc<T>(n, F->nnzV, &F->Vcp, &F->Vri, &F->Vval, st);
    if (e.code != DIAF_OK) {
        free_factors(F);
        return e;
    }
    if (F->vtri == 1 || F->vtri == -1) F->vtri = -F->vtri;
    F->left = 1;
    *out = F;
    return {};
}

template <class T>
Err solve_impl(diaf_ctx* ctx, const diaf_csc* A, diaf_factors* F, const T* b, T* x, double rtol,
               int maxit, diaf_solve_info* info)
{
    // With graphs on, the iterations run on a library stream (the caller's
    // may be the null stream, which cannot be captured): first wait for the
    // caller's work, then everything below is ordered on that stream and the
    // call returns after it has drained.
    const bool use_graph = ctx->opt_graph && F != nullptr;
    hipStream_t st = ctx->stream;
    if (use_graph) {
        if (!ctx->gstream) DIAF_HIP_TRY(hipStreamCreateWithFlags(&ctx->gstream, hipStreamNonBlocking));
        DIAF_TRY(sync(ctx->stream));
        st = ctx->gstream;
    }
    const int n = (int)A->n;
    auto t0 = std::chrono::steady_clock::now();
    if (F) {
        if (F->n != n || F->dtype != A->dtype) return {DIAF_EINVAL, "factors do not match A"};
        DIAF_TRY(ensure_apply<T>(ctx, F));
        if (F->stats.count_zero_pivot) {
            // the first preconditioner application would divide by zero
            DIAF_HIP_TRY(hipMemsetAsync(x, 0, sizeof(T) * n, st));
            DIAF_TRY(sync(st));
            info->iters = 1;
            info->flag = 3;
            info->relres = 1.0;
            info->relres_true = 1.0;
            info->ms = 0.0;
            return {};
        }
    }
    // CSR copy of A
    DevBlocks blocks;  // everything below is freed on every return path
    int32_t *rp = nullptr, *ci = nullptr;
    T* cv = nullptr;
    DIAF_TRY(dmalloc(&rp, sizeof(int32_t) * (n + 1)));
    blocks.keep(rp);
    DIAF_TRY(dmalloc(&ci, sizeof(int32_t) * (size_t)A->nnz));
    blocks.keep(ci);
    DIAF_TRY(dmalloc(&cv, sizeof(T) * (size_t)A->nnz));
    blocks.keep(cv);
    DIAF_TRY(csc_to_csr<T>(n, A->nnz, A->colptr, A->rowidx, (const T*)A->val, rp, ci, cv, st));
    // work vectors
    BicgVecs<T> V{};
    V.n = n;
    V.b = b;
    V.x = x;
    T* buf = nullptr;
    DIAF_TRY(dmalloc(&buf, sizeof(T) * (size_t)n * 8));
    blocks.keep(buf);
    V.r = buf; V.rh = buf + n; V.p = buf + 2 * (size_t)n; V.v = buf + 3 * (size_t)n;
    V.ph = buf + 4 * (size_t)n; V.s = buf + 5 * (size_t)n; V.sh = buf + 6 * (size_t)n;
    V.t = buf + 7 * (size_t)n;
    DIAF_TRY(dmalloc(&V.partial, sizeof(double) * 4 * 1024));
    blocks.keep(V.partial);
    DIAF_TRY(dmalloc(&V.st, sizeof(BicgState<T>)));
    blocks.keep(V.st);
    DIAF_HIP_TRY(hipMemsetAsync(V.st, 0, sizeof(BicgState<T>), st));
    const int32_t* done = &V.st->done;
    // Left preconditioning: BiCGSTAB on M A x = M b (the preconditioned
    // residual drives the iteration and the stop test); the products are
    // M (A p) and M (A s), and x advances along p and s themselves, so ph
    // and sh alias p and s.  The true residual at the end uses b itself.
    const bool left = F && F->left;
    T *bl = nullptr, *av = nullptr;
    struct FreeL {
        T** a; T** b;
        ~FreeL() { dfree(*a); dfree(*b); }
    } freel{&bl, &av};
    if (left) {
        DIAF_TRY(dmalloc(&bl, sizeof(T) * n));
        DIAF_TRY(dmalloc(&av, sizeof(T) * n));
        DIAF_TRY(enqueue_apply<T>(ctx, F, b, bl, nullptr, st));
        V.b = bl;
        V.ph = V.p;
        V.sh = V.s;
    }
    // Right preconditioning with a triangular V: the two solves of an
    // iteration write to buffers of their own, which the stage kernels after
    // them (bicg_alpha, bicg_xr) refill with the not-ready sentinel, so no
    // solve needs a fill launch (filled here once for the first iteration).
    const bool trsv_prec = !left && F && F->vtri != 0 && F->vtri != 3;
    T* tsolve = nullptr;
    if (trsv_prec) {
        DIAF_TRY(dmalloc(&tsolve, sizeof(T) * (size_t)n * 2));
        blocks.keep(tsolve);
        DIAF_TRY(launch_fill_sentinel<T>(n, tsolve, st));
        DIAF_TRY(launch_fill_sentinel<T>(n, tsolve + n, st));
        V.clr_a = tsolve;
        V.clr_x = tsolve + n;
    }
    const auto apply_prec = [&](const T* in, T* out, T* tbuf) -> Err {
        if (tbuf) return enqueue_apply_with<T>(ctx, F, in, out, done, st, tbuf, F->ctl, true);
        return enqueue_apply<T>(ctx, F, in, out, done, st);
    };
    DIAF_TRY(bicg_init<T>(V, rtol, maxit, st));
    BicgState<T> hs{};
    const int batch = (int)ctx->opt_batch;
    // one batch of iterations; every stage returns at once after convergence
    const auto enqueue_batch = [&]() -> Err {
        for (int q = 0; q < batch; ++q) {
            DIAF_TRY(bicg_update_p<T>(V, st));
            if (left) {
                DIAF_TRY(launch_spmv_csr<T>(n, A->nnz, rp, ci, cv, V.p, av, done, st));
                DIAF_TRY(enqueue_apply<T>(ctx, F, av, V.v, done, st));
                DIAF_TRY(bicg_alpha<T>(V, st));
                DIAF_TRY(bicg_s<T>(V, st));
                DIAF_TRY(launch_spmv_csr<T>(n, A->nnz, rp, ci, cv, V.s, av, done, st));
                DIAF_TRY(enqueue_apply<T>(ctx, F, av, V.t, done, st));
                DIAF_TRY(bicg_omega<T>(V, st));
                DIAF_TRY(bicg_xr<T>(V, st));
                continue;
            }
            if (F) DIAF_TRY(apply_prec(V.p, V.ph, V.clr_a));
            else DIAF_HIP_TRY(hipMemcpyAsync(V.ph, V.p, sizeof(T) * n, hipMemcpyDeviceToDevice, st));
            DIAF_TRY(launch_spmv_csr<T>(n, A->nnz, rp, ci, cv, V.ph, V.v, done, st));
            DIAF_TRY(bicg_alpha<T>(V, st));
            DIAF_TRY(bicg_s<T>(V, st));
            if (F) DIAF_TRY(apply_prec(V.s, V.sh, V.clr_x));
            else DIAF_HIP_TRY(hipMemcpyAsync(V.sh, V.s, sizeof(T) * n, hipMemcpyDeviceToDevice, st));
            DIAF_TRY(launch_spmv_csr<T>(n, A->nnz, rp, ci, cv, V.sh, V.t, done, st));
            DIAF_TRY(bicg_omega<T>(V, st));
            DIAF_TRY(bicg_xr<T>(V, st));
        }
        return {};
    };
    // captured once, replayed per batch (kernels only: no memset or copy
    // nodes).  The first batch is launched directly and the capture and
    // instantiation run on the host while the device works through it; the
    // kernels and their order are the same either way.
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    struct GraphFree {
        hipGraph_t* g; hipGraphExec_t* e;
        ~GraphFree() {
            if (*e) (void)hipGraphExecDestroy(*e);
            if (*g) (void)hipGraphDestroy(*g);
        }
    } gfree{&graph, &gexec};
    const auto capture = [&]() -> Err {
        DIAF_HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        Err e = enqueue_batch();
        hipGraph_t g = nullptr;
        const hipError_t ec = hipStreamEndCapture(st, &g);
        graph = g;
        DIAF_TRY(e);
        DIAF_HIP_TRY(ec);
        DIAF_HIP_TRY(hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0));
        return {};
    };
    for (int it0 = 0;; it0 += batch) {
        if (gexec) DIAF_HIP_TRY(hipGraphLaunch(gexec, st));
        else DIAF_TRY(enqueue_batch());
        if (use_graph && !gexec) DIAF_TRY(capture());
        DIAF_TRY(read1(V.st, &hs, st));
        if (F && (F->vtri == 1 || F->vtri == -1)) {
            TrsvCtl c{};
            DIAF_TRY(read1(F->ctl, &c, st));
            if (c.error) return {DIAF_EDEVICE, "triangular solve exceeded its wait budget"};
        }
        if (hs.done) break;
        if (it0 > maxit + batch) break;  // cannot happen: maxit stops the loop on the device
    }
    DIAF_TRY(bicg_half_fix<T>(V, st));
    DIAF_TRY(launch_spmv_csr<T>(n, A->nnz, rp, ci, cv, V.x, V.t, nullptr, st));
    V.b = b;
    DIAF_TRY(bicg_true_residual<T>(V, st));
    DIAF_TRY(read1(V.st, &hs, st));
    auto t1 = std::chrono::steady_clock::now();
    info->iters = hs.it;
    info->flag = hs.flag;
    info->relres = hs.res;
    info->relres_true = hs.tt;
    info->ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
    return {};
}

// Autotuner: times the candidate launch shapes on the caller's own problem
// and keeps the fastest in the context.  Factor: persistent grid of the
// one-wave kernel, then (when generic buckets occur) threads per column of
// the generic kernel, each by the factor kernels' event time (best of 2).
// Solve: graph replay, iterations per host poll and polling back-off, by the
// wall time per iteration of 32-iteration solves after a warm-up solve.
template <class T>
Err autotune_impl(diaf_ctx* ctx, const diaf_csc* A, const diaf_spec* spec, int mode)
{
    const int n = (int)A->n;
    int launches = 0;
    const auto time_factor = [&](double& best) -> Err {
        best = INFINITY;
        for (int rep = 0; rep < 2; ++rep) {
            diaf_factors* F = nullptr;
            DIAF_TRY(factor_impl<T>(ctx, A, spec, mode, &F));
            best = std::min(best, (double)F->stats.ms_factor_kernels);
            launches = F->stats.factor_launches;
            free_factors(F);
        }
        return {};
    };
    {
        const int grids[] = {1024, 2048, 4096, 8192, 16384};
        double best = INFINITY;
        int pick = 0;
        for (int g : grids) {
            ctx->ftune.small_grid = g;
            double ms;
            DIAF_TRY(time_factor(ms));
            if (ms < best) { best = ms; pick = g; }
        }
        ctx->ftune.small_grid = pick;
    }
    if (launches >= 2 || ctx->opt_generic_only || spec->gram_fp32) {
        double best = INFINITY;
        int pick = 0;
        for (int t = 0; t < kNumClassTables; ++t) {
            ctx->opt_class_table = t;
            double ms;
            DIAF_TRY(time_factor(ms));
            if (ms < best) { best = ms; pick = t; }
        }
        ctx->opt_class_table = pick;
    }
    if (launches >= 2 || ctx->opt_generic_only || spec->gram_fp32) {
        const int nts[] = {0, 64, 128, 256, 512};
        double best = INFINITY;
        int pick = 0;
        for (int t : nts) {
            ctx->ftune.generic_nt = t;
            double ms;
            DIAF_TRY(time_factor(ms));
            if (ms < best) { best = ms; pick = t; }
        }
        ctx->ftune.generic_nt = pick;
    }
    // solve
    diaf_factors* F = nullptr;
    DIAF_TRY(factor_impl<T>(ctx, A, spec, mode, &F));
    std::unique_ptr<diaf_factors, void (*)(diaf_factors*)> Fh(F, free_factors);
    T *b = nullptr, *x = nullptr;
    DIAF_TRY(dmalloc(&b, sizeof(T) * (size_t)n));
    DIAF_TRY(dmalloc(&x, sizeof(T) * (size_t)n));
    struct VFree {
        T** a; T** c;
        ~VFree() { dfree(*a); dfree(*c); }
    } vfree{&b, &x};
    {
        std::vector<T> ones((size_t)n, num<T>::one());
        DIAF_HIP_TRY(hipMemcpy(b, ones.data(), sizeof(T) * (size_t)n, hipMemcpyHostToDevice));
    }
    const auto time_solve = [&](int maxit, double& ms_per_it) -> Err {
        DIAF_HIP_TRY(hipMemsetAsync(x, 0, sizeof(T) * (size_t)n, ctx->stream));
        DIAF_TRY(sync(ctx->stream));
        diaf_solve_info info{};
        DIAF_TRY(solve_impl<T>(ctx, A, F, b, x, 1e-300, maxit, &info));
        ms_per_it = info.iters > 0 ? info.ms / info.iters : INFINITY;
        return {};
    };
    double warm;
    DIAF_TRY(time_solve(8, warm));  // the first apply builds the CSR copies
    {
        // waves per workgroup of the triangular solve
        double bw = INFINITY;
        int pw = ctx->trsv.waves;
        for (int w : {4, 8, 16}) {
            ctx->trsv.waves = w;
            double ms = INFINITY;
            for (int rep = 0; rep < 2; ++rep) {
                double t;
                DIAF_TRY(time_solve(32, t));
                ms = std::min(ms, t);
            }
            if (ms < bw) { bw = ms; pw = w; }
        }
        ctx->trsv.waves = pw;
    }
    double best = INFINITY;
    int pg = (int)ctx->opt_graph, pb = (int)ctx->opt_batch, po = ctx->trsv.backoff;
    for (int g = 0; g < 2; ++g)
        for (int bt : {8, 32})
            for (int bo = 0; bo < 2; ++bo) {
                ctx->opt_graph = g;
                ctx->opt_batch = bt;
                ctx->trsv.backoff = bo;
                double ms = INFINITY;
                for (int rep = 0; rep < 2; ++rep) {
                    double t;
                    DIAF_TRY(time_solve(32, t));
                    ms = std::min(ms, t);
                }
                if (ms < best) { best = ms; pg = g; pb = bt; po = bo; }
            }
    ctx->opt_graph = pg;
    ctx->opt_batch = pb;
    ctx->trsv.backoff = po;
    return {};
}

}  // namespace

extern "C" diaf_status diaf_solve(diaf_ctx* ctx, const diaf_csc* A, const diaf_factors* F,
                                  const void* b, void* x, double rtol, int32_t maxit,
                                  diaf_solve_info* info)
{
    if (!ctx) return DIAF_EINVAL;
    Err e = check_csc_host(A);
    if (e.code) return fail(ctx, e);
    if (!b || !x || !info) return fail(ctx, DIAF_EINVAL, "NULL argument");
    if (!(rtol > 0) || maxit < 1) return fail(ctx, DIAF_EINVAL, "rtol must be > 0 and maxit >= 1");
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, DIAF_EDEVICE, "hipSetDevice");
    auto* Fm = const_cast<diaf_factors*>(F);
    e = A->dtype == DIAF_F64
            ? solve_impl<double>(ctx, A, Fm, (const double*)b, (double*)x, rtol, maxit, info)
            : solve_impl<zc>(ctx, A, Fm, (const zc*)b, (zc*)x, rtol, maxit, info);
    if (e.code) return fail(ctx, e);
    if (info->flag == 1) return fail(ctx, DIAF_ENOCONV, "BiCGSTAB: no convergence within maxit");
    if (info->flag == 2) return fail(ctx, DIAF_EBREAKDOWN, "BiCGSTAB: breakdown");
    if (info->flag == 3) return fail(ctx, DIAF_ESINGULAR, "V has a zero or non-finite pivot");
    return DIAF_OK;
}

namespace {

// Persistent autotuning: one JSON object per line of the file, keyed by the
// device architecture and the problem's shape.
const char* const kTuneKeys[] = {"small_grid", "generic_nt", "class_table", "trsv_waves",
                                 "graph", "solve_batch", "trsv_backoff"};
constexpr int kNumTuneKeys = 7;

std::string tune_key(const diaf_ctx* ctx, const diaf_csc* A, const diaf_spec* spec, int mode)
{
    hipDeviceProp_t prop{};
    std::string arch = "unknown";
    if (hipGetDeviceProperties(&prop, ctx->device) == hipSuccess) arch = prop.gcnArchName;
    char buf[512];
    snprintf(buf, sizeof buf, "%s|%s|%s|n=%lld|nnz=%lld|w=%d:%d|v=%d:%d|left=%d|fp32=%d",
             arch.c_str(), mode == DIAF_UNIT_V ? "unit_v" : "unit_w",
             A->dtype == DIAF_C128 ? "c128" : "f64", (long long)A->n, (long long)A->nnz,
             (int)spec->w_kind, (int)spec->w_topk, (int)spec->v_kind, (int)spec->v_count,
             (int)spec->left, (int)spec->gram_fp32);
    return buf;
}

void tune_get(const diaf_ctx* ctx, int64_t* v)
{
    v[0] = ctx->ftune.small_grid;
    v[1] = ctx->ftune.generic_nt;
    v[2] = ctx->opt_class_table;
    v[3] = ctx->trsv.waves;
    v[4] = ctx->opt_graph;
    v[5] = ctx->opt_batch;
    v[6] = ctx->trsv.backoff;
}

// Reads the file (a missing file is empty).  Lines other than "{", "}" and
// entries written by tune_write are an error, so a foreign file is never
// overwritten.
Err tune_read(const char* path, std::vector<std::pair<std::string, std::vector<int64_t>>>& out)
{
    FILE* f = fopen(path, "r");
    if (!f) return {};
    char line[4096];
    int ln = 0;
    Err err{};
    while (fgets(line, sizeof line, f)) {
        ++ln;
        std::string t(line);
        while (!t.empty() && (t.back() == '\n' || t.back() == '\r' || t.back() == ' ')) t.pop_back();
        if (t.empty() || t == "{" || t == "}") continue;
        const size_t q0 = t.find('"'), q1 = q0 == std::string::npos ? q0 : t.find('"', q0 + 1);
        const size_t br = q1 == std::string::npos ? q1 : t.find('{', q1);
        if (q0 != 0 || br == std::string::npos) {
            err = {DIAF_EINVAL, std::string("tune file ") + path + ": unrecognised line " +
                                    std::to_string(ln)};
            break;
        }
        std::vector<int64_t> vals(kNumTuneKeys, INT64_MIN);
        for (int q = 0; q < kNumTuneKeys; ++q) {
            const std::string pat = std::string("\"") + kTuneKeys[q] + "\": ";
            const size_t p = t.find(pat, br);
            if (p != std::string::npos) vals[q] = strtoll(t.c_str() + p + pat.size(), nullptr, 10);
        }
        out.push_back({t.substr(q0 + 1, q1 - q0 - 1), vals});
    }
    fclose(f);
    return err;
}

Err tune_write(const char* path,
               const std::vector<std::pair<std::string, std::vector<int64_t>>>& entries)
{
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = fopen(tmp.c_str(), "w");
    if (!f) return {DIAF_EINVAL, std::string("tune file ") + path + ": cannot write"};
    fprintf(f, "{\n");
    for (size_t e = 0; e < entries.size(); ++e) {
        fprintf(f, "\"%s\": {", entries[e].first.c_str());
        for (int q = 0; q < kNumTuneKeys; ++q)
            fprintf(f, "%s\"%s\": %lld", q ? ", " : "", kTuneKeys[q],
                    (long long)entries[e].second[q]);
        fprintf(f, "}%s\n", e + 1 < entries.size() ? "," : "");
    }
    fprintf(f, "}\n");
    const bool ok = fclose(f) == 0;
    if (!ok || rename(tmp.c_str(), path) != 0)
        return {DIAF_EINVAL, std::string("tune file ") + path + ": cannot write"};
    return {};
}

}  // namespace

extern "C" diaf_status diaf_autotune_cached(diaf_ctx* ctx, const diaf_csc* A,
                                            const diaf_spec* spec, int32_t mode, const char* path,
                                            int32_t* from_cache)
{
    if (!ctx || !A || !spec || !path || !from_cache) return DIAF_EINVAL;
    *from_cache = 0;
    std::vector<std::pair<std::string, std::vector<int64_t>>> entries;
    Err e = tune_read(path, entries);
    if (e.code) return fail(ctx, e);
    const std::string key = tune_key(ctx, A, spec, mode);
    for (auto& en : entries) {
        if (en.first != key) continue;
        bool whole = true;
        for (int64_t v : en.second) whole = whole && v != INT64_MIN;
        if (!whole) break;
        for (int q = 0; q < kNumTuneKeys; ++q) {
            const diaf_status s = diaf_ctx_set_option(ctx, kTuneKeys[q], en.second[q]);
            if (s != DIAF_OK) return s;
        }
        *from_cache = 1;
        return DIAF_OK;
    }
    const diaf_status s = diaf_autotune(ctx, A, spec, mode);
    if (s != DIAF_OK) return s;
    std::vector<int64_t> vals(kNumTuneKeys);
    tune_get(ctx, vals.data());
    bool found = false;
    for (auto& en : entries)
        if (en.first == key) { en.second = vals; found = true; }
    if (!found) entries.push_back({key, vals});
    e = tune_write(path, entries);
    if (e.code) return fail(ctx, e);
    return DIAF_OK;
}

extern "C" diaf_status diaf_autotune(diaf_ctx* ctx, const diaf_csc* A, const diaf_spec* spec,
                                     int32_t mode)
{
    if (!ctx) return DIAF_EINVAL;
    Err e = check_csc_host(A);
    if (e.code) return fail(ctx, e);
    if (!spec) return fail(ctx, DIAF_EINVAL, "spec is NULL");
    e = check_spec(A, spec, mode);
    if (e.code) return fail(ctx, e);
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, DIAF_EDEVICE, "hipSetDevice");
    e = A->dtype == DIAF_F64 ? autotune_impl<double>(ctx, A, spec, mode)
                             : autotune_impl<zc>(ctx, A, spec, mode);
    if (e.code) return fail(ctx, e);
    return DIAF_OK;
}

// ===========================================================================
// Learned proposer entry points
// ===========================================================================
extern "C" {

diaf_status diaf_model_create(diaf_ctx* ctx, const float* params_host, diaf_model** out)
{
    if (!ctx) return DIAF_EINVAL;
    if (!params_host || !out) return fail(ctx, DIAF_EINVAL, "NULL argument");
    *out = nullptr;
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, DIAF_EDEVICE, "hipSetDevice");
    auto* m = new diaf_model;
    m->ctx = ctx;
    Err e;
    const size_t np = DIAF_MLP_NPARAM;
    if (!e.code) e = dmalloc(&m->params, sizeof(float) * np);
    if (!e.code) e = dmalloc(&m->m, sizeof(float) * np);
    if (!e.code) e = dmalloc(&m->v, sizeof(float) * np);
    if (!e.code) e = dmalloc(&m->grad, sizeof(float) * np);
    if (!e.code) e = dmalloc(&m->scratch, sizeof(float) * mlp_scratch_floats());
    if (!e.code) e = dmalloc(&m->loss, sizeof(double));
    if (!e.code) {
        hipError_t h = hipMemcpyAsync(m->params, params_host, sizeof(float) * np,
                                      hipMemcpyHostToDevice, ctx->stream);
        if (h == hipSuccess) h = hipMemsetAsync(m->m, 0, sizeof(float) * np, ctx->stream);
        if (h == hipSuccess) h = hipMemsetAsync(m->v, 0, sizeof(float) * np, ctx->stream);
        if (h == hipSuccess) h = hipStreamSynchronize(ctx->stream);
        if (h != hipSuccess) e = {DIAF_EDEVICE, hipGetErrorString(h)};
    }
    if (e.code) {
        diaf_model_destroy(m);
        return fail(ctx, e);
    }
    *out = m;
    return DIAF_OK;
}

diaf_status diaf_model_get_params(diaf_ctx* ctx, const diaf_model* m, float* params_host)
{
    if (!ctx) return DIAF_EINVAL;
    if (!m || !params_host) return fail(ctx, DIAF_EINVAL, "NULL argument");
    hipError_t h = hipMemcpyAsync(params_host, m->params, sizeof(float) * DIAF_MLP_NPARAM,
                                  hipMemcpyDeviceToHost, ctx->stream);
    if (h == hipSuccess) h = hipStreamSynchronize(ctx->stream);
    if (h != hipSuccess) return fail(ctx, DIAF_EDEVICE, hipGetErrorString(h));
    return DIAF_OK;
}

void diaf_model_destroy(diaf_model* m)
{
    if (!m) return;
    dfree(m->params); dfree(m->m); dfree(m->v); dfree(m->grad); dfree(m->scratch); dfree(m->loss);
    delete m;
}

diaf_status diaf_features(diaf_ctx* ctx, const diaf_csc* A, const diaf_pattern* C, float* feat)
{
    if (!ctx) return DIAF_EINVAL;
    Err e = check_csc_host(A);
    if (e.code) return fail(ctx, e);
    if (!C || !feat) return fail(ctx, DIAF_EINVAL, "NULL argument");
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, DIAF_EDEVICE, "hipSetDevice");
    e = validate_pattern(C, A->n, 0, "candidate pattern", ctx->stream);
    if (!e.code)
        e = A->dtype == DIAF_F64
                ? launch_features<double>((int)A->n, A->colptr, A->rowidx, (const double*)A->val,
                                          C->colptr, C->rowidx, feat, ctx->stream)
                : launch_features<zc>((int)A->n, A->colptr, A->rowidx, (const zc*)A->val,
                                      C->colptr, C->rowidx, feat, ctx->stream);
    if (!e.code) e = sync(ctx->stream);
    if (e.code) return fail(ctx, e);
    return DIAF_OK;
}

diaf_status diaf_labels(diaf_ctx* ctx, const diaf_csc* A, const diaf_factors* F, double tau,
                        float* labels)
{
    if (!ctx) return DIAF_EINVAL;
    Err e = check_csc_host(A);
    if (e.code) return fail(ctx, e);
    if (!F || !labels) return fail(ctx, DIAF_EINVAL, "NULL argument");
    if (F->n != A->n || F->dtype != A->dtype) return fail(ctx, DIAF_EINVAL, "factors do not match A");
    e = A->dtype == DIAF_F64
            ? launch_labels<double>((int)A->n, A->colptr, A->rowidx, (const double*)A->val, F->Jcp,
                                    F->Jri, (const double*)F->Wval, tau, labels, ctx->stream)
            : launch_labels<zc>((int)A->n, A->colptr, A->rowidx, (const zc*)A->val, F->Jcp, F->Jri,
                                (const zc*)F->Wval, tau, labels, ctx->stream);
    if (!e.code) e = sync(ctx->stream);
    if (e.code) return fail(ctx, e);
    return DIAF_OK;
}

diaf_status diaf_mlp_forward(diaf_ctx* ctx, const diaf_model* m, const float* feat, int64_t npairs,
                             float* scores)
{
    if (!ctx) return DIAF_EINVAL;
    if (!m || (!feat && npairs) || (!scores && npairs) || npairs < 0)
        return fail(ctx, DIAF_EINVAL, "bad argument");
    Err e = launch_mlp_forward(m->params, feat, npairs, scores, ctx->stream);
    if (!e.code) e = sync(ctx->stream);
    if (e.code) return fail(ctx, e);
    return DIAF_OK;
}

diaf_status diaf_mlp_loss_grad(diaf_ctx* ctx, const diaf_model* mc, const float* feat,
                               const float* labels, int64_t npairs, float* grad, double* loss_host)
{
    if (!ctx) return DIAF_EINVAL;
    if (!mc || !feat || !labels || npairs <= 0 || !loss_host) return fail(ctx, DIAF_EINVAL, "bad argument");
    auto* m = const_cast<diaf_model*>(mc);
    Err e = launch_mlp_loss_grad(m->params, feat, labels, npairs, grad ? grad : m->grad, m->loss,
                                 m->scratch, ctx->stream);
    if (!e.code) e = read1(m->loss, loss_host, ctx->stream);
    if (e.code) return fail(ctx, e);
    return DIAF_OK;
}

diaf_status diaf_mlp_train_step(diaf_ctx* ctx, diaf_model* m, const float* feat,
                                const float* labels, int64_t npairs, float lr, double* loss_host)
{
    if (!ctx) return DIAF_EINVAL;
    if (!m || !feat || !labels || npairs <= 0 || !(lr > 0)) return fail(ctx, DIAF_EINVAL, "bad argument");
    Err e = launch_mlp_loss_grad(m->params, feat, labels, npairs, m->grad, m->loss, m->scratch,
                                 ctx->stream);
    if (!e.code) e = launch_adam(m->params, m->grad, m->m, m->v, ++m->step, lr, ctx->stream);
    if (!e.code && loss_host) e = read1(m->loss, loss_host, ctx->stream);
    if (e.code) return fail(ctx, e);
    return DIAF_OK;
}

}  // extern "C"
