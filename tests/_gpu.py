"""Helpers of the GPU parity tests: run the HIP library through the C ABI and
compare with the CPU oracle on the same seeded inputs."""
from __future__ import annotations

import sys

import numpy as np

import oracle

EPS = np.finfo(np.float64).eps

# Residual bar: |r_gpu - r_oracle| <= 1e-10 r_oracle + 1e-12 s_j with the
# column scale s_j = 1 + ||B_j||_F ||w_j|| (unit-norm v) or ||B_j||_F
# (unit-norm w).  The relative term binds wherever the residual is resolved;
# the floor covers numerically exact columns (r ~ 1e-13 s_j), where the
# residual is first order in the rounding of the singular vector and the
# QR route and the Gram route land on different rounding-level values.
# Only at such a near-exact column (r_oracle <= 1e-8 sqrt(gap) s_j) may the
# residual also use what the angle bar allows: with the singular vector
# within an angle theta of the optimum, r^2 = r_opt^2 + gap theta^2 to first
# order (gap = the oracle's relative squared singular gap), so with r_opt ~ 0
# r is first order in theta, and theta <= ANGLE_TOL allows
# ANGLE_TOL sqrt(gap) s_j.  Elsewhere r is stationary in theta and gets no
# such allowance.
# A gap-degenerate column (the oracle's flag: gap < 1e-6) has no angle bar:
# its optimal vector is not determined to 1e-8.  Every unit vector in the
# span of the two extreme singular vectors attains r^2 <= r_opt^2 + gap S^2
# (S = sigma_1(M_j) <= 1 for unit-norm v, sigma_max <= ||B_j||_F for unit-norm
# w), with equality for the second singular vector, so there the GPU's
# residual must lie between r_opt - tol and (1 + 1e-6) times that bound
# plus tol (the factor covers the oracle's rounding of the tiny gap): the
# GPU's column is then as good as some vector of the degenerate subspace.
# Such columns are counted.
RES_REL = 1e-10
RES_FLOOR = 1e-12
ANGLE_TOL = 1e-8
# Flags that both sides must set identically (column by column), except on
# columns the oracle marks as lying within a factor 100 of a rank threshold
# (RANK_EDGE) or whose |v_jj| / ||v_j|| is within 1 % of the 1e-2 threshold.
AGREE = (oracle.RANK_DEFICIENT | oracle.SMALL_DIAG | oracle.TIE_EDGE | oracle.STABILIZED
         | oracle.NO_DIAG_ROW | oracle.NULL_CHOICE)


def angle_excluded(flags, mode):
    """The oracle's flags that make the singular vector not unique to 1e-8:
    a degenerate gap, a rank test at its threshold, or (unit-norm v) a rank
    deficient B, whose least-squares solution is not unique.  A unit-norm-w
    column with a null space keeps the angle check: its w is fixed by the
    null-space choice (or is the only null vector)."""
    ex = oracle.GAP_DEGENERATE | oracle.RANK_EDGE
    if mode == "unit_v":
        ex |= oracle.RANK_DEFICIENT
    return (int(flags) & ex) != 0


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def oracle_pattern(A, w, wtopk=0):
    if w == "A":
        return oracle.pattern_A(A)
    if w == "A2":
        return oracle.pattern_A2(A)
    if w == "A_1hop_topk":
        return oracle.pattern_1hop(A, wtopk)
    raise KeyError(w)


def run_gpu(ctx, A, w, v, vcount, mode, wtopk=0, gram_fp32=False, dA=None):
    from paper_1208_3573_amd import diaf
    if dA is None:
        dA = diaf.DeviceCSC.from_host(A)
    spec = diaf.make_spec(w=w, v=v, v_count=vcount, w_topk=wtopk, gram_fp32=gram_fp32)
    F = diaf.diaf_factor(ctx, dA, spec, mode)
    return F, F.to_host(), dA


def block_fro(A, J):
    """||A(:, J_j)||_F for every column j."""
    cn2 = np.zeros(A.n)
    np.add.at(cn2, np.repeat(np.arange(A.n), np.diff(A.colptr)), np.abs(A.val) ** 2)
    per = cn2[J.rowidx]
    out = np.zeros(A.n)
    np.add.at(out, np.repeat(np.arange(A.n), np.diff(J.colptr)), per)
    return np.sqrt(out)


def sin_angle(x, y):
    x = np.asarray(x).ravel()
    y = np.asarray(y).ravel()
    ny = np.vdot(y, y).real
    nx = np.linalg.norm(x)
    if ny == 0 or nx == 0:
        return 0.0 if ny == nx else 1.0
    return float(np.linalg.norm(x - y * (np.vdot(y, x) / ny)) / nx)


def compare(H, J, O, A, mode, cols=None, check_pattern=True, stab_tol=1e-2):
    """Compare GPU factors H (to_host dict) with oracle factors O on columns
    `cols` (all when None).  Returns a summary; asserts the bars: identical
    V patterns; residuals within the bar above; singular vectors within
    ANGLE_TOL except where the oracle's flags exclude them; the flags of
    AGREE equal on both sides; GPU-only gap flags only where the oracle's
    gap is below 1e-4."""
    n = A.n
    if check_pattern:
        assert np.array_equal(H["Wcp"], J.colptr), "W pattern colptr differs"
        assert np.array_equal(H["Wri"], J.rowidx), "W pattern rows differ"
    cols = np.arange(n) if cols is None else np.asarray(cols)
    bn = block_fro(A, J)
    worst_res = 0.0
    worst_ang = 0.0
    excluded = 0
    floor_only = 0
    gap_floor = 0
    degenerate_res = 0
    flag_edge = 0
    gap_gpu_only = 0
    gap_orc_only = 0
    vpat_bad = []
    res_bad = []
    ang_bad = []
    flag_bad = []
    for j in cols:
        g_rows = H["Vri"][H["Vcp"][j]:H["Vcp"][j + 1]]
        g_vals = H["Vval"][H["Vcp"][j]:H["Vcp"][j + 1]]
        lo = O.lcount[j]
        o_rows = O.Vrows_pad[j, :lo]
        o_vals = O.Vvals_pad[j, :lo]
        of = int(O.flags[j])
        gf = int(H["flags"][j])
        # flag agreement
        on = np.linalg.norm(o_vals)
        dpos = np.flatnonzero(o_rows == j)
        ratio = abs(o_vals[dpos[0]]) / on if dpos.size and on > 0 else 0.0
        near = (of & oracle.RANK_EDGE) or abs(ratio - 1e-2) <= 1e-4 or \
            abs(ratio - stab_tol) <= 1e-2 * stab_tol
        # bits that follow from a non-unique vector (|v_jj|, the tie band of
        # the seed's scores) are not compared on gap-degenerate columns
        agree = AGREE if not of & oracle.GAP_DEGENERATE else \
            (oracle.RANK_DEFICIENT | oracle.NO_DIAG_ROW | oracle.NULL_CHOICE)
        if near:
            flag_edge += 1
        elif (gf ^ of) & agree:
            flag_bad.append((int(j), gf, of))
        if (gf & ~of) & oracle.GAP_DEGENERATE:
            gap_gpu_only += 1
            if not O.gap[j] < 1e-4:
                flag_bad.append((int(j), gf, of, float(O.gap[j])))
        if (of & ~gf) & oracle.GAP_DEGENERATE:
            gap_orc_only += 1
        if not np.array_equal(g_rows, o_rows):
            vpat_bad.append(j)
            continue
        wsl = slice(J.colptr[j], J.colptr[j + 1])
        g_w = H["Wval"][wsl]
        o_w = O.Wval[wsl]
        s = bn[j] if mode == "unit_w" else 1.0 + bn[j] * np.linalg.norm(o_w)
        tol = RES_REL * O.r[j] + RES_FLOOR * s
        d = abs(H["r"][j] - O.r[j])
        worst_res = max(worst_res, d / max(tol, 1e-300))
        if d > RES_REL * O.r[j]:
            floor_only += 1
        if of & oracle.GAP_DEGENERATE and not d <= tol:
            S = 1.0 if mode == "unit_v" else bn[j]
            # the bound is attained by the second singular vector itself; the
            # factor 1 + 1e-6 covers the oracle's rounding of a gap this small
            hi = np.sqrt(O.r[j] ** 2 + max(O.gap[j], 0.0) * S * S) * (1 + 1e-6) + tol
            if O.r[j] - tol <= H["r"][j] <= hi:
                degenerate_res += 1
            else:
                res_bad.append((int(j), float(H["r"][j]), float(O.r[j]), float(tol),
                                float(O.gap[j]), "degenerate"))
        elif not d <= tol:
            allow = ANGLE_TOL * np.sqrt(max(O.gap[j], 0.0)) * s
            if O.r[j] <= allow and d <= tol + allow:
                gap_floor += 1
            else:
                res_bad.append((int(j), float(H["r"][j]), float(O.r[j]), float(tol),
                                float(O.gap[j])))
        if angle_excluded(of, mode):
            excluded += 1
            continue
        a = sin_angle(g_vals, o_vals) if mode == "unit_v" else sin_angle(g_w, o_w)
        worst_ang = max(worst_ang, a)
        if not a <= ANGLE_TOL:
            ang_bad.append((int(j), a))
    summ = dict(cols=len(cols), excluded=excluded, floor_only=floor_only, gap_floor=gap_floor,
                degenerate_res=degenerate_res, flag_edge=flag_edge, gap_gpu_only=gap_gpu_only, gap_orc_only=gap_orc_only,
                worst_res_over_tol=worst_res,
                worst_angle=worst_ang, vpattern_mismatch=len(vpat_bad),
                null_choice=int(np.sum((O.flags[cols] & oracle.NULL_CHOICE) != 0)),
                gpu_tie_edge=int(np.sum((H["flags"][cols] & oracle.TIE_EDGE) != 0)))
    say("parity:", summ)
    assert not vpat_bad, f"V pattern differs in columns {vpat_bad[:10]}"
    assert not res_bad, f"residual outside the bar: {res_bad[:5]}"
    assert not ang_bad, f"singular vector angle above {ANGLE_TOL}: {ang_bad[:5]}"
    assert not flag_bad, f"flags differ (column, gpu, oracle): {flag_bad[:5]}"
    return summ
