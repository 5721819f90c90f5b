/*
 * CPU FP64 oracle for the direct approximate factoring AW ~ V
 * (Byckling & Huhtanen).  TEST INFRASTRUCTURE ONLY: called by the tests,
 * the smoke check and the benchmark's CPU-baseline leg, never by the GPU
 * library.  Built with gcc -O2 -ffp-contract=off -fopenmp.
 *
 * This file holds the integer (pattern) work, the top-k rule for the V
 * pattern, and instantiates the type-generic column solvers, apply and
 * BiCGSTAB of oracle_scalar.inc for double and double complex.
 */
#include "oracle_common.h"

int orc_cmp_i32(const void* a, const void* b)
{
    int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
    return (x > y) - (x < y);
}

typedef struct { double s; int32_t idx; } orc_si;

static int cmp_score_desc(const void* a, const void* b)
{
    const orc_si* x = (const orc_si*)a;
    const orc_si* y = (const orc_si*)b;
    if (x->s > y->s) return -1;
    if (x->s < y->s) return 1;
    return (x->idx > y->idx) - (x->idx < y->idx);
}

/*
 * Optimal V pattern for a fixed w (Section 3.1: among the admissible rows
 * keep those that make the retained part of A w_j largest): the q
 * candidates with the largest scores.  Candidates are listed in ascending
 * row order.  Exact ties, and scores within a relative 1e-10 of the q-th
 * largest score s*, form one tie class that is filled in ascending row
 * order; scores above s*(1 + 1e-10) are always taken.  *edge is set when a
 * score lies within 1e-12 s* of a band boundary.  Returns the number of
 * chosen candidates, written to out in ascending row order.
 */
int orc_select_topk(int nc, const int32_t* cand, const double* score, int q, int32_t* out,
                    int* edge)
{
    *edge = 0;
    if (q <= 0) return 0;
    if (nc <= q) {
        for (int t = 0; t < nc; ++t) out[t] = cand[t];
        return nc;
    }
    orc_si* tmp = (orc_si*)malloc(sizeof(orc_si) * (size_t)nc);
    for (int t = 0; t < nc; ++t) { tmp[t].s = score[t]; tmp[t].idx = t; }
    qsort(tmp, (size_t)nc, sizeof(orc_si), cmp_score_desc);
    double sstar = tmp[q - 1].s;
    free(tmp);
    double hi = sstar * (1.0 + 1e-10), lo = sstar * (1.0 - 1e-10);
    int cnt = 0;
    for (int t = 0; t < nc; ++t)
        if (score[t] > hi) out[cnt++] = cand[t];
    for (int t = 0; t < nc && cnt < q; ++t)
        if (score[t] >= lo && score[t] <= hi) out[cnt++] = cand[t];
    for (int t = 0; t < nc; ++t) {
        double d1 = fabs(score[t] - hi), d2 = fabs(score[t] - lo);
        if (sstar > 0.0 && (d1 <= 1e-12 * sstar || d2 <= 1e-12 * sstar)) *edge = 1;
    }
    qsort(out, (size_t)cnt, sizeof(int32_t), orc_cmp_i32);
    return cnt;
}

/*
 * W pattern = pattern(A^2) taken symbolically (no cancellation): column j
 * is the union of the row sets of the columns A(:, c), c in rows(A(:, j)).
 * This is the truncated Neumann series of Section 4.1 with diagonal V_0,
 * truncation k = 2 and no dropping.  Two-call protocol: with Jri == NULL
 * only Jcp (n+1) is filled.
 */
int orc_pattern_a2(int n, const int32_t* Acp, const int32_t* Ari, int32_t* Jcp, int32_t* Jri)
{
    int32_t* mk = (int32_t*)calloc((size_t)n, sizeof(int32_t));
    int32_t* out = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    if (!mk || !out) return -2;
    if (!Jri) Jcp[0] = 0;
    for (int j = 0; j < n; ++j) {
        int cnt = 0;
        for (int p = Acp[j]; p < Acp[j + 1]; ++p) {
            int c = Ari[p];
            for (int q = Acp[c]; q < Acp[c + 1]; ++q) {
                int i = Ari[q];
                if (!mk[i]) { mk[i] = 1; out[cnt++] = i; }
            }
        }
        qsort(out, (size_t)cnt, sizeof(int32_t), orc_cmp_i32);
        if (Jri) memcpy(Jri + Jcp[j], out, sizeof(int32_t) * (size_t)cnt);
        else Jcp[j + 1] = Jcp[j] + cnt;
        for (int t = 0; t < cnt; ++t) mk[out[t]] = 0;
    }
    free(mk); free(out);
    return 0;
}

/* ---- real instantiation ---- */
#define T double
#define SFX(name) name##_d
#define CONJ(x) (x)
#define RE(x) (x)
#define IMP(x) (0.0)
#define MK2(re, im) (re)
#define ABS2(x) ((x) * (x))
#define ABS(x) fabs(x)
#define ABSR(x) fabs(x)
#include "oracle_scalar.inc"
#undef T
#undef SFX
#undef CONJ
#undef RE
#undef IMP
#undef MK2
#undef ABS2
#undef ABS
#undef ABSR

/* ---- complex instantiation ---- */
#define T double complex
#define SFX(name) name##_z
#define CONJ(x) conj(x)
#define RE(x) creal(x)
#define IMP(x) cimag(x)
#define MK2(re, im) CMPLX(re, im)
#define ABS2(x) (creal(x) * creal(x) + cimag(x) * cimag(x))
#define ABS(x) sqrt(creal(x) * creal(x) + cimag(x) * cimag(x))
#define ABSR(x) cabs(x)
#include "oracle_scalar.inc"
#undef T
#undef SFX
#undef CONJ
#undef RE
#undef IMP
#undef MK2
#undef ABS2
#undef ABS
#undef ABSR
