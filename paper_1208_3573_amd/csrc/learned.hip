// Learned W-pattern proposer: features of (column j, candidate i) pairs of
// the A^2 candidate pattern, labels from a plain factorization, an MLP
// 16 -> 64 -> 64 -> 1 (ReLU) with forward, loss/gradient and Adam kernels,
// and the proposal J_j = {j} U {i : score >= 0}.
//
// Features use only column access to A (the paper's requirement): for the
// pair (j, i), with |.| the modulus, d_c = |a_cc|, s_c = sum_{r != c} |a_rc|,
// nrm_c = ||A(:,c)||, deg_c = nnz(A(:,c)), and the A^2 path statistics over
// c in rows(A(:,j)): pw = sum_c |a_ic||a_cj|, cnt = #{c : a_ic a_cj != 0},
// mx = max_c |a_ic||a_cj|:
//   f0 [i == j]          f1 [a_ij != 0]        f2 pw / max_col pw
//   f3 cnt / max_col cnt f4 |a_ij| / d_j       f5 deg_j / 8
//   f6 deg_i / 8         f7 d_j / (d_j + s_j)  f8 d_i / (d_i + s_i)
//   f9 sign(i - j)       f10 log2(1 + |i-j|)/24 f11 nrm_i / nrm_j
//   f12 mx / pw          f13 pw / (d_i d_j)    f14 |C_j| / 32
//   f15 fraction of the column's candidates with a larger pw
// computed in FP64 and stored as FP32.
#include "dcommon.h"
#include "factor_kernels.h"

namespace diaf {

static constexpr int NF = 16, NH = 64;
static constexpr int P_W1 = 0, P_B1 = P_W1 + NH * NF, P_W2 = P_B1 + NH, P_B2 = P_W2 + NH * NH,
                     P_W3 = P_B2 + NH, P_B3 = P_W3 + NH, NPARAM = P_B3 + 1;

// ---------------------------------------------------------------------------
// Per-column scalars: d_c, s_c, nrm_c, deg_c.
// ---------------------------------------------------------------------------
template <class T>
__global__ void colstats_kernel(int n, const int32_t* Acp, const int32_t* Ari, const T* Aval,
                                double* d, double* s, double* nrm)
{
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    double dd = 0, ss = 0, n2 = 0;
    for (int p = Acp[c]; p < Acp[c + 1]; ++p) {
        double a = num<T>::abs(Aval[p]);
        n2 += a * a;
        if (Ari[p] == c) dd = a; else ss += a;
    }
    d[c] = dd;
    s[c] = ss;
    nrm[c] = sqrt(n2);
}

template <class T>
__device__ inline double entry_abs(const int32_t* Acp, const int32_t* Ari, const T* Aval, int row,
                                   int col)
{
    int lo = Acp[col], hi = Acp[col + 1] - 1;
    while (lo <= hi) {
        int mid = (lo + hi) >> 1;
        int r = Ari[mid];
        if (r == row) return num<T>::abs(Aval[mid]);
        if (r < row) lo = mid + 1; else hi = mid - 1;
    }
    return 0.0;
}

template <class T>
__device__ inline void path_stats(const int32_t* Acp, const int32_t* Ari, const T* Aval, int j, int i,
                                  double& pw, int& cnt, double& mx)
{
    pw = 0; cnt = 0; mx = 0;
    for (int p = Acp[j]; p < Acp[j + 1]; ++p) {
        double pr = entry_abs(Acp, Ari, Aval, i, Ari[p]) * num<T>::abs(Aval[p]);
        pw += pr;
        if (pr != 0.0) ++cnt;
        mx = fmax(mx, pr);
    }
}

static constexpr int FCMAX = 512;  // candidates per column kept in LDS for the rank feature

// One wave per column.
template <class T>
__global__ void __launch_bounds__(64) features_kernel(int n, const int32_t* Acp, const int32_t* Ari,
                                                     const T* Aval, const int32_t* Ccp,
                                                     const int32_t* Cri, const double* d,
                                                     const double* s, const double* nrm,
                                                     float* feat)
{
    __shared__ double spw[FCMAX];
    const int j = blockIdx.x;
    const int lane = threadIdx.x;
    const int cb = Ccp[j], nc = Ccp[j + 1] - cb;
    // column maxima
    double pwmax = 0;
    int cntmax = 0;
    for (int t = lane; t < nc; t += 64) {
        double pw, mx;
        int cnt;
        path_stats(Acp, Ari, Aval, j, Cri[cb + t], pw, cnt, mx);
        if (t < FCMAX) spw[t] = pw;
        pwmax = fmax(pwmax, pw);
        cntmax = max(cntmax, cnt);
    }
    for (int o = 32; o > 0; o >>= 1) {
        pwmax = fmax(pwmax, __shfl_xor(pwmax, o));
        cntmax = max(cntmax, __shfl_xor(cntmax, o));
    }
    __syncthreads();
    const double dj = d[j], sj = s[j], nj = nrm[j];
    const int degj = Acp[j + 1] - Acp[j];
    for (int t = lane; t < nc; t += 64) {
        int i = Cri[cb + t];
        double pw, mx;
        int cnt;
        path_stats(Acp, Ari, Aval, j, i, pw, cnt, mx);
        int larger = 0;
        for (int u = 0; u < nc; ++u) {
            double pu;
            if (u < FCMAX) {
                pu = spw[u];
            } else {
                double mu;
                int cu;
                path_stats(Acp, Ari, Aval, j, Cri[cb + u], pu, cu, mu);
            }
            larger += (u != t) && (pu > pw);
        }
        double aij = entry_abs(Acp, Ari, Aval, i, j);
        bool inA = false;
        {
            int lo = Acp[j], hi = Acp[j + 1] - 1;
            while (lo <= hi) {
                int mid = (lo + hi) >> 1;
                if (Ari[mid] == i) { inA = true; break; }
                if (Ari[mid] < i) lo = mid + 1; else hi = mid - 1;
            }
        }
        double di = d[i], si = s[i];
        float* f = feat + (size_t)(cb + t) * NF;
        f[0] = i == j ? 1.f : 0.f;
        f[1] = inA ? 1.f : 0.f;
        f[2] = (float)(pwmax > 0 ? pw / pwmax : 0.0);
        f[3] = (float)(cntmax > 0 ? (double)cnt / cntmax : 0.0);
        f[4] = (float)(dj > 0 ? aij / dj : 0.0);
        f[5] = (float)(degj / 8.0);
        f[6] = (float)((Acp[i + 1] - Acp[i]) / 8.0);
        f[7] = (float)(dj + sj > 0 ? dj / (dj + sj) : 0.0);
        f[8] = (float)(di + si > 0 ? di / (di + si) : 0.0);
        f[9] = i > j ? 1.f : (i < j ? -1.f : 0.f);
        f[10] = (float)(log2(1.0 + fabs((double)i - (double)j)) / 24.0);
        f[11] = (float)(nj > 0 ? nrm[i] / nj : 0.0);
        f[12] = (float)(pw > 0 ? mx / pw : 0.0);
        f[13] = (float)(di > 0 && dj > 0 ? pw / (di * dj) : 0.0);
        f[14] = (float)(nc / 32.0);
        f[15] = (float)(nc > 1 ? (double)larger / (nc - 1) : 0.0);
    }
}

template <class T>
Err launch_features(int n, const int32_t* Acp, const int32_t* Ari, const T* Aval,
                    const int32_t* Ccp, const int32_t* Cri, float* feat, hipStream_t st)
{
    if (n == 0) return {};
    double* buf = nullptr;
    DIAF_TRY(amalloc((void**)&buf, sizeof(double) * 3 * (size_t)n, st));
    hipLaunchKernelGGL(colstats_kernel<T>, dim3((n + 255) / 256), dim3(256), 0, st, n, Acp, Ari,
                       Aval, buf, buf + n, buf + 2 * (size_t)n);
    hipLaunchKernelGGL(features_kernel<T>, dim3(n), dim3(64), 0, st, n, Acp, Ari, Aval, Ccp, Cri,
                       buf, buf + n, buf + 2 * (size_t)n, feat);
    DIAF_HIP_TRY(hipGetLastError());
    afree(buf, st);
    return {};
}

// ---------------------------------------------------------------------------
// Labels: 1 when |w_j(i)| ||A(:,i)|| >= tau max over the column, and i == j.
// ---------------------------------------------------------------------------
template <class T>
__global__ void __launch_bounds__(64) labels_kernel(int n, const int32_t* Jcp, const int32_t* Jri,
                                                   const T* Wval, const double* nrm, double tau,
                                                   float* labels)
{
    const int j = blockIdx.x;
    const int lane = threadIdx.x;
    const int b = Jcp[j], k = Jcp[j + 1] - b;
    double mxv = 0;
    for (int t = lane; t < k; t += 64) mxv = fmax(mxv, num<T>::abs(Wval[b + t]) * nrm[Jri[b + t]]);
    for (int o = 32; o > 0; o >>= 1) mxv = fmax(mxv, __shfl_xor(mxv, o));
    for (int t = lane; t < k; t += 64) {
        int i = Jri[b + t];
        double c = num<T>::abs(Wval[b + t]) * nrm[i];
        labels[b + t] = (i == j || c >= tau * mxv) ? 1.f : 0.f;
    }
}

template <class T>
Err launch_labels(int n, const int32_t* Acp, const int32_t* Ari, const T* Aval, const int32_t* Jcp,
                  const int32_t* Jri, const T* Wval, double tau, float* labels, hipStream_t st)
{
    if (n == 0) return {};
    double* buf = nullptr;
    DIAF_TRY(amalloc((void**)&buf, sizeof(double) * 3 * (size_t)n, st));
    hipLaunchKernelGGL(colstats_kernel<T>, dim3((n + 255) / 256), dim3(256), 0, st, n, Acp, Ari,
                       Aval, buf, buf + n, buf + 2 * (size_t)n);
    hipLaunchKernelGGL(labels_kernel<T>, dim3(n), dim3(64), 0, st, n, Jcp, Jri, Wval,
                       buf + 2 * (size_t)n, tau, labels);
    DIAF_HIP_TRY(hipGetLastError());
    afree(buf, st);
    return {};
}

// ---------------------------------------------------------------------------
// MLP forward: one thread per pair.  The parameters are read at indices
// the same for every lane, so they come in through scalar loads and enter
// the FMAs as scalar operands: no LDS traffic per multiply-add.  The
// multiply-adds run in the same order as in the gradient kernel.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) mlp_forward_kernel(const float* __restrict__ params,
                                                        const float* __restrict__ feat,
                                                        int64_t npairs, float* __restrict__ scores)
{
    // one pair per thread and no loop around it, so the weights are not
    // hoisted into registers for the whole kernel
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < npairs) {
        float x[NF];
        const float4* f4 = (const float4*)(feat + p * NF);
#pragma unroll
        for (int q = 0; q < NF / 4; ++q) {
            float4 v = f4[q];
            x[4 * q] = v.x; x[4 * q + 1] = v.y; x[4 * q + 2] = v.z; x[4 * q + 3] = v.w;
        }
        float h1[NH];
#pragma unroll
        for (int o = 0; o < NH; ++o) {
            float a = params[P_B1 + o];
#pragma unroll
            for (int q = 0; q < NF; ++q) a = fmaf(params[P_W1 + o * NF + q], x[q], a);
            h1[o] = fmaxf(a, 0.f);
        }
        float sc = params[P_B3];
        for (int o = 0; o < NH; ++o) {
            float a = params[P_B2 + o];
#pragma unroll
            for (int q = 0; q < NH; ++q) a = fmaf(params[P_W2 + o * NH + q], h1[q], a);
            sc = fmaf(params[P_W3 + o], fmaxf(a, 0.f), sc);
        }
        scores[p] = sc;
    }
}

Err launch_mlp_forward(const float* params, const float* feat, int64_t npairs, float* scores,
                       hipStream_t st)
{
    if (npairs <= 0) return {};
    const int64_t blocks = (npairs + 255) / 256;
    if (blocks > 0x7fffffffll) return {DIAF_EUNSUPPORTED, "MLP forward: too many pairs"};
    hipLaunchKernelGGL(mlp_forward_kernel, dim3((unsigned)blocks), dim3(256), 0, st, params, feat,
                       npairs, scores);
    DIAF_HIP_TRY(hipGetLastError());
    return {};
}

// ---------------------------------------------------------------------------
// Loss and gradient: mean binary cross-entropy with logits.  Persistent
// blocks of 128 threads take tiles of 128 pairs (one pair per thread),
// stage activations in LDS and accumulate the parameter gradient of their
// tiles; each block writes one partial gradient (and loss), reduced in a
// fixed order afterwards.
// ---------------------------------------------------------------------------
static constexpr int GT = 128;   // pairs per tile = threads per block
static constexpr int GBLK = 256; // persistent blocks
static constexpr int NPT = (NPARAM + GT - 1) / GT;  // parameters owned per thread

__global__ void __launch_bounds__(GT) mlp_grad_kernel(const float* params, const float* feat,
                                                    const float* labels, int64_t npairs,
                                                    float* partial, double* loss_partial)
{
    __shared__ float P[NPARAM];
    __shared__ float sA[GT][NH + 1];  // h1, later Delta1
    __shared__ float sB[GT][NH + 1];  // Delta2
    __shared__ float sC[GT][NH + 1];  // h2 (post-ReLU), later x
    __shared__ float sD[GT];          // delta3
    for (int q = threadIdx.x; q < NPARAM; q += GT) P[q] = params[q];
    __syncthreads();
    const int tid = threadIdx.x;
    float g[NPT];
#pragma unroll
    for (int u = 0; u < NPT; ++u) g[u] = 0.f;
    double lsum = 0.0;
    const float invN = 1.0f / (float)npairs;
    const int64_t ntiles = (npairs + GT - 1) / GT;
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int64_t p = tile * GT + tid;
        const bool valid = p < npairs;
        float x[NF];
#pragma unroll
        for (int q = 0; q < NF; ++q) x[q] = valid ? feat[p * NF + q] : 0.f;
        float h1[NH];
#pragma unroll
        for (int o = 0; o < NH; ++o) {
            float a = P[P_B1 + o];
#pragma unroll
            for (int q = 0; q < NF; ++q) a = fmaf(P[P_W1 + o * NF + q], x[q], a);
            h1[o] = fmaxf(a, 0.f);
            sA[tid][o] = h1[o];
        }
        float sc = P[P_B3];
        for (int o = 0; o < NH; ++o) {
            float a = P[P_B2 + o];
#pragma unroll
            for (int q = 0; q < NH; ++q) a = fmaf(P[P_W2 + o * NH + q], h1[q], a);
            float h2 = fmaxf(a, 0.f);
            sC[tid][o] = h2;
            sc = fmaf(P[P_W3 + o], h2, sc);
        }
        float d3 = 0.f;
        if (valid) {
            float y = labels[p];
            // loss = max(s,0) - s y + log(1 + exp(-|s|)); dloss/ds = sigmoid(s) - y
            lsum += (double)(fmaxf(sc, 0.f) - sc * y + log1pf(expf(-fabsf(sc))));
            float sg = 1.f / (1.f + expf(-sc));
            d3 = (sg - y) * invN;
        }
        sD[tid] = d3;
        // Delta2 = d3 w3 [h2 > 0]
#pragma unroll
        for (int o = 0; o < NH; ++o) sB[tid][o] = sC[tid][o] > 0.f ? d3 * P[P_W3 + o] : 0.f;
        __syncthreads();
        // gradients of w3, b3, W2, b2 (this thread's parameters)
#pragma unroll
        for (int u = 0; u < NPT; ++u) {
            int q = tid + u * GT;
            if (q < P_W2 || q >= NPARAM) continue;
            float acc = 0.f;
            if (q < P_B2) {            // W2[o][k] : sum Delta2_o h1_k
                int o = (q - P_W2) / NH, k = (q - P_W2) % NH;
                for (int r = 0; r < GT; ++r) acc = fmaf(sB[r][o], sA[r][k], acc);
            } else if (q < P_W3) {     // b2[o]
                int o = q - P_B2;
                for (int r = 0; r < GT; ++r) acc += sB[r][o];
            } else if (q < P_B3) {     // w3[o] : sum d3 h2_o
                int o = q - P_W3;
                for (int r = 0; r < GT; ++r) acc = fmaf(sD[r], sC[r][o], acc);
            } else {                   // b3
                for (int r = 0; r < GT; ++r) acc += sD[r];
            }
            g[u] += acc;
        }
        __syncthreads();
        // Delta1 = (W2^T Delta2) [h1 > 0]  -> sA ; x -> sC
        {
            float d2[NH];
#pragma unroll
            for (int o = 0; o < NH; ++o) d2[o] = sB[tid][o];
            for (int k = 0; k < NH; ++k) {
                float a = 0.f;
#pragma unroll
                for (int o = 0; o < NH; ++o) a = fmaf(P[P_W2 + o * NH + k], d2[o], a);
                sA[tid][k] = h1[k] > 0.f ? a : 0.f;
            }
#pragma unroll
            for (int q = 0; q < NF; ++q) sC[tid][q] = x[q];
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < NPT; ++u) {
            int q = tid + u * GT;
            if (q >= P_W2) continue;
            float acc = 0.f;
            if (q < P_B1) {            // W1[o][f] : sum Delta1_o x_f
                int o = q / NF, f = q % NF;
                for (int r = 0; r < GT; ++r) acc = fmaf(sA[r][o], sC[r][f], acc);
            } else {                   // b1[o]
                int o = q - P_B1;
                for (int r = 0; r < GT; ++r) acc += sA[r][o];
            }
            g[u] += acc;
        }
        __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < NPT; ++u) {
        int q = tid + u * GT;
        if (q < NPARAM) partial[(size_t)blockIdx.x * NPARAM + q] = g[u];
    }
    // loss partial (fixed-order block sum)
    __shared__ double sl[GT];
    sl[tid] = lsum;
    __syncthreads();
    if (tid == 0) {
        double t = 0;
        for (int r = 0; r < GT; ++r) t += sl[r];
        loss_partial[blockIdx.x] = t;
    }
}

__global__ void grad_reduce_kernel(const float* partial, int nblk, int64_t npairs, float* grad,
                                   const double* loss_partial, double* loss)
{
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < NPARAM) {
        float s = 0.f;
        for (int b = 0; b < nblk; ++b) s += partial[(size_t)b * NPARAM + q];
        grad[q] = s;
    }
    if (q == 0) {
        double t = 0;
        for (int b = 0; b < nblk; ++b) t += loss_partial[b];
        *loss = t / (double)npairs;
    }
}

Err launch_mlp_loss_grad(const float* params, const float* feat, const float* labels,
                         int64_t npairs, float* grad, double* loss_dev, float* scratch,
                         hipStream_t st)
{
    if (npairs <= 0) return {DIAF_EINVAL, "npairs must be positive"};
    int64_t ntiles = (npairs + GT - 1) / GT;
    int nblk = (int)(ntiles < GBLK ? ntiles : GBLK);
    double* lp = (double*)(scratch + (size_t)GBLK * NPARAM);
    hipLaunchKernelGGL(mlp_grad_kernel, dim3(nblk), dim3(GT), 0, st, params, feat, labels, npairs,
                       scratch, lp);
    hipLaunchKernelGGL(grad_reduce_kernel, dim3((NPARAM + 255) / 256), dim3(256), 0, st, scratch,
                       nblk, npairs, grad, lp, loss_dev);
    DIAF_HIP_TRY(hipGetLastError());
    return {};
}

size_t mlp_scratch_floats() { return (size_t)GBLK * NPARAM + 2 * GBLK + 16; }

__global__ void adam_kernel(float* params, const float* grad, float* m, float* v, int step,
                            float lr)
{
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= NPARAM) return;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    float g = grad[q];
    float mq = b1 * m[q] + (1.f - b1) * g;
    float vq = b2 * v[q] + (1.f - b2) * g * g;
    m[q] = mq;
    v[q] = vq;
    float mh = mq / (1.f - powf(b1, (float)step));
    float vh = vq / (1.f - powf(b2, (float)step));
    params[q] -= lr * mh / (sqrtf(vh) + eps);
}

Err launch_adam(float* params, const float* grad, float* m, float* v, int step, float lr,
                hipStream_t st)
{
    hipLaunchKernelGGL(adam_kernel, dim3((NPARAM + 255) / 256), dim3(256), 0, st, params, grad, m, v,
                       step, lr);
    DIAF_HIP_TRY(hipGetLastError());
    return {};
}

// ---------------------------------------------------------------------------
// Proposal: J_j = {j} U {i in C_j : score >= 0} (sigmoid >= 1/2).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(64) proposal_kernel(int n, const int32_t* Ccp, const int32_t* Cri,
                                                     const float* scores, int32_t* cnt,
                                                     const int32_t* Jcp, int32_t* Jri)
{
    const int j = blockIdx.x;
    const int lane = threadIdx.x;
    const int b = Ccp[j], k = Ccp[j + 1] - b;
    int base = 0;
    for (int t0 = 0; t0 < k; t0 += 64) {
        int t = t0 + lane;
        bool keep = false;
        if (t < k) keep = (Cri[b + t] == j) || (scores[b + t] >= 0.f);
        uint64_t mask = __ballot(keep);
        if (Jri && keep) {
            int pos = base + __popcll(mask & ((1ull << lane) - 1ull));
            Jri[Jcp[j] + pos] = Cri[b + t];
        }
        base += __popcll(mask);
    }
    if (!Jri && lane == 0) cnt[j] = base;
}

Err launch_pattern_from_scores(int n, const int32_t* Ccp, const int32_t* Cri, const float* scores,
                               int32_t* cnt, const int32_t* Jcp, int32_t* Jri, hipStream_t st)
{
    if (n == 0) return {};
    hipLaunchKernelGGL(proposal_kernel, dim3(n), dim3(64), 0, st, n, Ccp, Cri, scores, cnt, Jcp, Jri);
    DIAF_HIP_TRY(hipGetLastError());
    return {};
}

// ---------------------------------------------------------------------------
// Residual-gated fallback: columns with fb[j] != 0 take the candidate
// pattern C_j; the others keep J_j and their already computed W values.
// ---------------------------------------------------------------------------
__global__ void fallback_count_kernel(int n, const int32_t* Jcp, const int32_t* Ccp,
                                      const uint8_t* fb, int32_t* cnt)
{
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n) cnt[j] = fb[j] ? Ccp[j + 1] - Ccp[j] : Jcp[j + 1] - Jcp[j];
}

template <class T>
__global__ void fallback_fill_kernel(int n, const int32_t* Jcp, const int32_t* Jri, const T* Wval,
                                     const int32_t* Ccp, const int32_t* Cri, const uint8_t* fb,
                                     const int32_t* Jcp2, int32_t* Jri2, T* Wval2, uint32_t* flags)
{
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    int o = Jcp2[j];
    if (fb[j]) {
        for (int p = Ccp[j]; p < Ccp[j + 1]; ++p) { Jri2[o] = Cri[p]; Wval2[o] = num<T>::zero(); ++o; }
        flags[j] |= DIAF_FLAG_FELL_BACK;
    } else {
        for (int p = Jcp[j]; p < Jcp[j + 1]; ++p) { Jri2[o] = Jri[p]; Wval2[o] = Wval[p]; ++o; }
    }
}

Err launch_fallback_count(int n, const int32_t* Jcp, const int32_t* Ccp, const uint8_t* fb,
                          int32_t* cnt, hipStream_t st)
{
    hipLaunchKernelGGL(fallback_count_kernel, dim3((n + 255) / 256), dim3(256), 0, st, n, Jcp, Ccp,
                       fb, cnt);
    DIAF_HIP_TRY(hipGetLastError());
    return {};
}

template <class T>
Err launch_fallback_fill(int n, const int32_t* Jcp, const int32_t* Jri, const T* Wval,
                         const int32_t* Ccp, const int32_t* Cri, const uint8_t* fb,
                         const int32_t* Jcp2, int32_t* Jri2, T* Wval2, uint32_t* flags,
                         hipStream_t st)
{
    hipLaunchKernelGGL(fallback_fill_kernel<T>, dim3((n + 255) / 256), dim3(256), 0, st, n, Jcp,
                       Jri, Wval, Ccp, Cri, fb, Jcp2, Jri2, Wval2, flags);
    DIAF_HIP_TRY(hipGetLastError());
    return {};
}

template Err launch_fallback_fill<double>(int, const int32_t*, const int32_t*, const double*,
                                          const int32_t*, const int32_t*, const uint8_t*,
                                          const int32_t*, int32_t*, double*, uint32_t*, hipStream_t);
template Err launch_fallback_fill<zc>(int, const int32_t*, const int32_t*, const zc*,
                                      const int32_t*, const int32_t*, const uint8_t*,
                                      const int32_t*, int32_t*, zc*, uint32_t*, hipStream_t);
template Err launch_features<double>(int, const int32_t*, const int32_t*, const double*,
                                     const int32_t*, const int32_t*, float*, hipStream_t);
template Err launch_features<zc>(int, const int32_t*, const int32_t*, const zc*, const int32_t*,
                                 const int32_t*, float*, hipStream_t);
template Err launch_labels<double>(int, const int32_t*, const int32_t*, const double*,
                                   const int32_t*, const int32_t*, const double*, double, float*,
                                   hipStream_t);
template Err launch_labels<zc>(int, const int32_t*, const int32_t*, const zc*, const int32_t*,
                               const int32_t*, const zc*, double, float*, hipStream_t);

}  // namespace diaf
