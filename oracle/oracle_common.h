/*
 * CPU FP64 oracle for the direct approximate factoring AW ~ V
 * (Byckling & Huhtanen, "Preconditioning with direct approximate factoring
 * of the inverse").  TEST INFRASTRUCTURE ONLY: the tests, the smoke check
 * and the benchmark's CPU baseline call it; the GPU library never does.
 * Plain, slow, obviously-correct loops; no code is shared with the GPU
 * library.
 *
 * Shared declarations for the type-generic part (oracle_scalar.inc) and the
 * integer/pattern part (oracle.c).
 */
#ifndef ORACLE_COMMON_H
#define ORACLE_COMMON_H

#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Per-column flag bits reported by the oracle. */
#define ORC_RANK_DEFICIENT 1u  /* B_j (DIAF-Q) or B_j minus rows L_j (DIAF-S) numerically rank deficient */
#define ORC_GAP_DEGENERATE 2u  /* extreme singular value not separated: vector not unique */
#define ORC_SMALL_DIAG 4u      /* |v_jj| < 1e-2 ||v_j|| */
#define ORC_TIE_EDGE 16u       /* a top-k score lies at the edge of the tie band */
#define ORC_STABILIZED 32u     /* v_j replaced by the constrained solution of Section 3.2 */
#define ORC_NO_DIAG_ROW 64u    /* row j does not occur in the shadow R_j */
#define ORC_NULL_CHOICE 128u   /* unit-norm w chosen in a null space of dimension >= 2 */
#define ORC_RANK_EDGE 256u     /* a rank test quantity within a factor 100 of its threshold */

/* V pattern rules. */
enum { ORC_V_EXPLICIT = 0, ORC_V_DIAG = 1, ORC_V_GS_UPPER = 2, ORC_V_GS_LOWER = 3,
       ORC_V_TOPK_UPPER = 4, ORC_V_TOPK_LOWER = 5, ORC_V_LEV_UPPER = 6, ORC_V_LEV_LOWER = 7,
       ORC_V_TOPK_BLOCK = 8 };
/* Norm modes: unit-norm columns of V (first basic algorithm, DIAF-Q) or of
 * W (second basic algorithm, DIAF-S). */
enum { ORC_UNIT_V = 0, ORC_UNIT_W = 1 };

int orc_select_topk(int nc, const int32_t* cand, const double* score, int q,
                    int32_t* out, int* edge);
int orc_cmp_i32(const void* a, const void* b);

#endif
