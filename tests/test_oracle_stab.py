"""Pins of the oracle's constrained computation of Section 3.2 (unit-norm v,
triangular V): when |v_jj| < tol ||v_j||, v_jj := r and the other rows S of
L_j carry e^{i theta} v^, v^ the top right singular vector of M^ (the columns
of Q^* at S), theta the argument of the first component of U^* p (p the
column of Q^* at row j); w_j is the least-squares solution for that v.

Every check uses NumPy's QR / SVD / least squares on the dense A(:, J_j), not
the oracle's Householder QR and one-sided Jacobi, or a property the paper
states (the direction of v^ does not depend on r).
"""
import numpy as np
import pytest

import oracle
import synth
from tests._dense import Aj, cols_of, dense, v_of, w_of

R = 2.0


def _case(cplx, per_col=4, seed=0, n=400):
    return synth.random_small(n, per_col, seed, complex_=cplx)


def _q(Ad, J, j):
    """Orthonormal basis of range(A_j) (n x k) by NumPy's QR."""
    return np.linalg.qr(Aj(Ad, J, j), mode="reduced")[0]


def _vfull(n, rows, vals, dt):
    v = np.zeros(n, dtype=dt)
    v[rows] = vals
    return v


@pytest.mark.parametrize("cplx", [False, True])
def test_stab_l1_is_scaled_spai(cplx):
    """l = 1 (diagonal V) with every column constrained: v_j = r e_j and w_j
    the least-squares solution of A_j w = r e_j (r times the sparse
    approximate inverse column of Example 3.2)."""
    A = _case(cplx)
    Ad = dense(A)
    J = oracle.pattern_A(A)
    F = oracle.factor(A, J, "unit_v", "diag", stab_r=R, stab_tol=1.1)
    assert np.all(F.flags & 32)
    for j in range(A.n):
        rows, vals = v_of(F, j)
        assert list(rows) == [j] and abs(vals[0] - R) == 0.0
        _, w = w_of(F, j)
        e = np.zeros(A.n, dtype=Ad.dtype)
        e[j] = R
        wref = np.linalg.lstsq(Aj(Ad, J, j), e, rcond=None)[0]
        assert np.linalg.norm(w - wref) <= 1e-11 * np.linalg.norm(wref)


@pytest.mark.parametrize("cplx", [False, True])
def test_stab_l2_closed_form(cplx):
    """|S| = 1: M^ is one column m of Q^*, so v^ is a unimodular scalar and
    the first component of U^* p is m^* p / ||m||; hence v_s = H_sj / |H_sj|
    with H = Q Q^* (the projector onto range(A_j))."""
    A = _case(cplx)
    Ad = dense(A)
    J = oracle.pattern_A(A)
    F = oracle.factor(A, J, "unit_v", "topk_lower", 2, stab_r=R, stab_tol=1.1)
    checked = 0
    for j in range(A.n):
        rows, vals = v_of(F, j)
        if len(rows) != 2:
            continue
        assert F.flags[j] & 32
        s = rows[0] if rows[1] == j else rows[1]
        Q = _q(Ad, J, j)
        hsj = Q[s] @ Q[j].conj()
        if abs(hsj) < 1e-12:
            continue
        vs = vals[list(rows).index(s)]
        vj = vals[list(rows).index(j)]
        assert vj == R
        assert abs(vs - hsj / abs(hsj)) <= 1e-11
        v = _vfull(A.n, rows, vals, Ad.dtype)
        wref = np.linalg.lstsq(Aj(Ad, J, j), v, rcond=None)[0]
        _, w = w_of(F, j)
        assert np.linalg.norm(w - wref) <= 1e-10 * np.linalg.norm(wref)
        checked += 1
    assert checked > 50


@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("vrule,vcount", [("topk_lower", 5), ("topk_upper", 4), ("gs_upper", 0)])
def test_stab_top_singular_vector_and_best_phase(cplx, vrule, vcount):
    """On the columns the rule constrains: v_jj = r, ||v_S|| = 1, ||M^ v_S||
    equals the largest singular value of M^ (NumPy SVD), and no other phase
    e^{i phi} v_S gives a larger ||Q^* v|| = ||r p + M^ v^|| (brute force over
    phases; for real data the only other phase is -1).  The properties hold
    for any constrained column, so a looser trigger (0.2) gives more cases."""
    A = _case(cplx)
    Ad = dense(A)
    J = oracle.pattern_A2(A)
    F = oracle.factor(A, J, "unit_v", vrule, vcount, stab_r=R, stab_tol=0.2)
    cols = np.nonzero(F.flags & 32)[0]
    assert len(cols) >= 3
    phis = np.linspace(0.0, 2 * np.pi, 73)[1:-1] if cplx else np.array([np.pi])
    for j in cols:
        rows, vals = v_of(F, j)
        d = list(rows).index(j)
        assert vals[d] == R
        S = [t for t in range(len(rows)) if t != d]
        if not S:
            continue
        vS = vals[S]
        assert abs(np.linalg.norm(vS) - 1.0) <= 1e-12
        Q = _q(Ad, J, j)
        Mh = Q[rows[S]].conj().T  # columns of Q^* at the rows S
        smax = np.linalg.svd(Mh, compute_uv=False)[0]
        assert abs(np.linalg.norm(Mh @ vS) - smax) <= 1e-10 * max(1.0, smax)
        v = _vfull(A.n, rows, vals, Ad.dtype)
        best = np.linalg.norm(Q.conj().T @ v)
        for phi in phis:
            vv = v.copy()
            vv[rows[S]] = np.exp(1j * phi) * vS if cplx else -vS
            assert np.linalg.norm(Q.conj().T @ vv) <= best * (1 + 1e-12)


def test_stab_direction_independent_of_r():
    """The paper notes that the solution does not depend on r_j > 0: the
    entries on S coincide for r = 1 and r = 2."""
    A = _case(True)
    J = oracle.pattern_A2(A)
    F1 = oracle.factor(A, J, "unit_v", "topk_lower", 5, stab_r=1.0)
    F2 = oracle.factor(A, J, "unit_v", "topk_lower", 5, stab_r=2.0)
    cols = np.nonzero(F2.flags & 32)[0]
    assert len(cols) >= 3
    assert np.array_equal(np.nonzero(F1.flags & 32)[0], cols)
    for j in cols:
        r1, v1 = v_of(F1, j)
        r2, v2 = v_of(F2, j)
        assert np.array_equal(r1, r2)
        off = r1 != j
        assert np.max(np.abs(v1[off] - v2[off])) <= 1e-12
        assert v1[~off][0] == 1.0 and v2[~off][0] == 2.0


@pytest.mark.parametrize("cplx", [False, True])
def test_stab_residual_closed_form(cplx):
    """r_j = ||A w_j - v_j|| (computed directly by the oracle) equals
    sqrt(||v||^2 - ||Q^* v||^2) for the least-squares w (Appendix A.1)."""
    A = _case(cplx)
    Ad = dense(A)
    J = oracle.pattern_A2(A)
    F = oracle.factor(A, J, "unit_v", "topk_lower", 5, stab_r=R)
    cols = np.nonzero(F.flags & 32)[0]
    assert len(cols) >= 3
    for j in cols:
        rows, vals = v_of(F, j)
        v = _vfull(A.n, rows, vals, Ad.dtype)
        Q = _q(Ad, J, j)
        rc = np.sqrt(max(0.0, np.vdot(v, v).real - np.linalg.norm(Q.conj().T @ v) ** 2))
        assert abs(F.r[j] - rc) <= 1e-10 * max(1.0, rc)


def test_stab_triggers_exactly_on_small_diagonals():
    """The constrained columns are the ones the plain computation flags
    with |v_jj| < 1e-2 ||v_j|| (and only those); unit-norm w and explicit
    V patterns are left alone; elsewhere the factors are unchanged."""
    A = _case(False, per_col=4, seed=1)
    J = oracle.pattern_A(A)
    F0 = oracle.factor(A, J, "unit_v", "topk_lower", 5)
    F1 = oracle.factor(A, J, "unit_v", "topk_lower", 5, stab_r=R)
    small = np.nonzero(F0.flags & 4)[0]
    assert len(small) >= 3
    assert np.array_equal(np.nonzero(F1.flags & 32)[0], small)
    assert not np.any(F1.flags & 4)
    keep = np.setdiff1d(np.arange(A.n), small)
    for j in keep:
        assert np.array_equal(v_of(F0, j)[1], v_of(F1, j)[1])
        assert np.array_equal(w_of(F0, j)[1], w_of(F1, j)[1])
    Fw = oracle.factor(A, J, "unit_w", "topk_lower", 5, stab_r=R)
    assert not np.any(Fw.flags & 32)
    Vexp = oracle.pattern_A(A)
    Fe = oracle.factor(A, J, "unit_v", "explicit", Vexp=Vexp, stab_r=R, stab_tol=1.1)
    assert not np.any(Fe.flags & 32)
