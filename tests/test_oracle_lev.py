"""Pins of the oracle's V rule of Section 3.1: L_j = {j} plus the l_j - 1
admissible rows i whose columns of Q_j^* have the largest norm, i.e. the
largest sqrt(h_i) with h_i = (A_j (A_j^* A_j)^{-1} A_j^*)_{ii}, the diagonal
of the projector onto range(A_j).

The leverages are computed here from NumPy's least squares / pseudo-inverse
on the dense A(:, J_j), not from the oracle's Householder QR, and the
selection is redone with an independent sort (ties within 1e-10 relative go
to the lower row, as for the other top-k rule).
"""
import itertools

import numpy as np
import pytest

import oracle
import synth
from tests._dense import Aj, dense, v_of


def _leverage(Ad, J, j):
    A_j = Aj(Ad, J, j)
    P = A_j @ np.linalg.pinv(A_j)
    return np.sqrt(np.maximum(np.real(np.diag(P)), 0.0))


def _select(scores, rows, q):
    """Top q rows by score with the 1e-10 tie band filled by ascending row."""
    if q <= 0:
        return []
    if len(rows) <= q:
        return sorted(rows)
    s = np.sort(scores)[::-1][q - 1]
    hi, lo = s * (1 + 1e-10), s * (1 - 1e-10)
    inn = [r for r, sc in zip(rows, scores) if sc > hi]
    tie = sorted(r for r, sc in zip(rows, scores) if lo <= sc <= hi)
    return sorted(inn + tie[: q - len(inn)])


@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("tri", ["lower", "upper"])
def test_leverage_rule_pattern(cplx, tri):
    A = synth.random_small(120, 4, 3, complex_=cplx, diag_shift=1.0)
    Ad = dense(A)
    J = oracle.pattern_A2(A)
    l = 4
    F = oracle.factor(A, J, "unit_v", f"lev_{tri}", l)
    for j in range(A.n):
        lev = _leverage(Ad, J, j)
        support = np.nonzero(np.any(Aj(Ad, J, j) != 0, axis=1))[0]
        adm = [i for i in support if (i > j if tri == "lower" else i < j)]
        want = sorted([j] + _select(lev[adm], adm, l - 1))
        rows, _ = v_of(F, j)
        assert list(rows) == want, (j, list(rows), want)


def test_leverage_rule_maximises_frobenius_norm():
    """Section 3.1: the l - 1 admissible columns of Q_j^* with the largest
    norms give the submatrix M_j of the largest Frobenius norm (brute force
    over every subset on small columns)."""
    A = synth.random_small(40, 3, 4, diag_shift=1.0)
    Ad = dense(A)
    J = oracle.pattern_A(A)
    l = 3
    F = oracle.factor(A, J, "unit_v", "lev_lower", l)
    checked = 0
    for j in range(A.n):
        lev = _leverage(Ad, J, j)
        support = np.nonzero(np.any(Aj(Ad, J, j) != 0, axis=1))[0]
        adm = [i for i in support if i > j]
        if len(adm) < l:
            continue
        rows, _ = v_of(F, j)
        chosen = [i for i in rows if i != j]
        f_chosen = np.sum(lev[chosen] ** 2)
        best = max(np.sum(lev[list(c)] ** 2) for c in itertools.combinations(adm, l - 1))
        assert f_chosen >= best * (1 - 1e-12)
        checked += 1
    assert checked >= 5


def test_leverage_rule_solution_is_the_unit_v_optimum():
    """On the rows the rule picks, v_j is the top right singular vector of
    M_j (checked through the closed form r_j^2 = 1 - sigma_1(M_j)^2 with M_j
    from NumPy's QR) and the constrained variant of Section 3.2 applies to
    the rule like to the other triangular rules."""
    A = synth.random_small(200, 4, 0)
    Ad = dense(A)
    J = oracle.pattern_A(A)
    F = oracle.factor(A, J, "unit_v", "lev_lower", 5)
    for j in range(0, A.n, 7):
        rows, _ = v_of(F, j)
        Q = np.linalg.qr(Aj(Ad, J, j), mode="reduced")[0]
        s1 = np.linalg.svd(Q[rows], compute_uv=False)[0]
        assert abs(F.r[j] - np.sqrt(max(0.0, 1 - s1 ** 2))) <= 1e-10
    Fs = oracle.factor(A, J, "unit_v", "lev_lower", 5, stab_r=2.0)
    small = np.nonzero(F.flags & oracle.SMALL_DIAG)[0]
    assert np.array_equal(np.nonzero(Fs.flags & oracle.STABILIZED)[0], small)
