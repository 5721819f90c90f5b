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
# QR route and the Gram route land on different rounding-level values.  The
# number of columns that pass only through the floor is reported.  A column
# that misses this bar is retried against the residual that the angle bar
# itself allows: with the singular vector within an angle theta of the
# optimum, r^2 = r_opt^2 + gap theta^2 to first order (gap = the relative
# squared singular gap, the oracle's), so near an exact column (r_opt ~ 0) r
# is first order in theta, and theta <= ANGLE_TOL allows ANGLE_TOL sqrt(gap)
# s_j.  Such columns are counted and reported.
RES_REL = 1e-10
RES_FLOOR = 1e-12
ANGLE_TOL = 1e-8
EXCLUDE = oracle.RANK_DEFICIENT | oracle.GAP_DEGENERATE


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


def compare(H, J, O, A, mode, cols=None, check_pattern=True):
    """Compare GPU factors H (to_host dict) with oracle factors O on columns
    `cols` (all when None).  Returns a summary; asserts the bars."""
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
    vpat_bad = []
    res_bad = []
    ang_bad = []
    for j in cols:
        g_rows = H["Vri"][H["Vcp"][j]:H["Vcp"][j + 1]]
        g_vals = H["Vval"][H["Vcp"][j]:H["Vcp"][j + 1]]
        lo = O.lcount[j]
        o_rows = O.Vrows_pad[j, :lo]
        o_vals = O.Vvals_pad[j, :lo]
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
        if not d <= tol:
            if d <= tol + ANGLE_TOL * np.sqrt(max(O.gap[j], 0.0)) * s:
                gap_floor += 1
            else:
                res_bad.append((int(j), float(H["r"][j]), float(O.r[j]), float(tol),
                                float(O.gap[j])))
        if (int(H["flags"][j]) | int(O.flags[j])) & EXCLUDE:
            excluded += 1
            continue
        a = sin_angle(g_vals, o_vals) if mode == "unit_v" else sin_angle(g_w, o_w)
        worst_ang = max(worst_ang, a)
        if not a <= ANGLE_TOL:
            ang_bad.append((int(j), a))
    summ = dict(cols=len(cols), excluded=excluded, floor_only=floor_only, gap_floor=gap_floor,
                worst_res_over_tol=worst_res,
                worst_angle=worst_ang, vpattern_mismatch=len(vpat_bad),
                gpu_tie_edge=int(np.sum((H["flags"][cols] & oracle.TIE_EDGE) != 0)))
    say("parity:", summ)
    assert not vpat_bad, f"V pattern differs in columns {vpat_bad[:10]}"
    assert not res_bad, f"residual outside the bar: {res_bad[:5]}"
    assert not ang_bad, f"singular vector angle above {ANGLE_TOL}: {ang_bad[:5]}"
    return summ
