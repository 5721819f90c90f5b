"""Pins of the oracle's per-column flags, the phase rule's fallback branch and
the null-space reading of the second basic algorithm.

Every expected value comes from NumPy (LAPACK QR and SVD, null spaces),
brute force over unit vectors, or a construction whose answer is known in
closed form; none re-runs the oracle's own routines.

Readings pinned here (Section 2.2 with Theorem 2.1; the paper assumes a
unique minimiser and is silent on the rest):
* rank-deficient: unit-norm v when |R_aa|^2 <= 1e-14 max_a ||B(:,a)||^2 for
  the QR of B = A(R_j, J_j) (or k > m); unit-norm w when
  sigma_min(Ahat)^2 <= 1e-14 ||Ahat||_F^2, Ahat = B without the rows L_j
  (or m - l < k);
* gap-degenerate: relative squared singular gap below 1e-6, of M_j = the
  rows L_j of Q (unit v) or of Ahat across the boundary of its null space
  (unit w);
* null-space choice: with a null space N of Ahat of dimension >= 2, w is
  the unit vector of N that maximises |(B w)_j|, i.e. P_N b^* / ||P_N b^*||;
* phase: v_jj real positive, or, when |v_jj| < 1e-8 ||v_j|| (or j not in
  L_j), the entry of largest modulus real positive, lowest row on ties.
"""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

import oracle
import synth
from tests._dense import cols_of, dense, sin_angle, v_of, w_of


def _csc(Ad):
    return synth.CSC.from_scipy(sp.csc_matrix(Ad))


def _pattern(lists, n):
    cp = np.cumsum([0] + [len(x) for x in lists]).astype(np.int32)
    ri = np.array([r for x in lists for r in sorted(x)], dtype=np.int32)
    return oracle.Pattern(n, cp, ri)


def _block(Ad, J, j):
    """Shadow rows R_j (ascending) and the dense block B = A(R_j, J_j)."""
    cj = cols_of(J, j)
    R = np.flatnonzero(np.any(Ad[:, cj] != 0, axis=1))
    return R, Ad[np.ix_(R, cj)]


def _complex_unit_grid_2():
    """Unit vectors of C^2 up to a global phase: (cos t, sin t e^{i p})."""
    t = np.linspace(0, np.pi / 2, 401)
    p = np.linspace(0, 2 * np.pi, 801)[:-1]
    T, P = np.meshgrid(t, p, indexing="ij")
    return np.stack([np.cos(T).ravel() + 0j, (np.sin(T) * np.exp(1j * P)).ravel()], axis=1)


def _fib_sphere(npts):
    i = np.arange(npts) + 0.5
    phi = np.arccos(1 - 2 * i / npts)
    th = np.pi * (1 + 5 ** 0.5) * i
    return np.stack([np.cos(th) * np.sin(phi), np.sin(th) * np.sin(phi), np.cos(phi)], axis=1)


# ---------------------------------------------------------------------------
# Null-space choice of the second basic algorithm.  With the full W pattern
# and L_j of size d, Ahat = A without d rows has a d-dimensional null space
# (A nonsingular); the oracle's w must beat every grid point of that null
# space in |(A w)_j| and sit at the grid's best point.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("cplx,d", [(False, 2), (False, 3), (True, 2)])
def test_null_choice_against_brute_force(cplx, d):
    n = 8
    rng = np.random.default_rng(40 + d + 10 * cplx)
    Ad = rng.standard_normal((n, n)) + 3 * np.eye(n)
    if cplx:
        Ad = Ad + 1j * rng.standard_normal((n, n))
    A = _csc(Ad)
    full = _pattern([list(range(n))] * n, n)
    Vexp = _pattern([sorted({j} | {(j + t) % n for t in range(1, d)}) for j in range(n)], n)
    F = oracle.factor(A, full, "unit_w", "explicit", Vexp=Vexp)
    if d == 2 and not cplx:
        grid = np.stack([np.cos(np.linspace(0, np.pi, 200001)),
                         np.sin(np.linspace(0, np.pi, 200001))], axis=1)
        hres = np.pi / 200000
    elif d == 3:
        grid = _fib_sphere(400000)
        hres = 2.0 * np.sqrt(4 * np.pi / 400000)
    else:
        grid = _complex_unit_grid_2()
        hres = np.pi / 800
    for j in range(n):
        L, v = v_of(F, j)
        _, w = w_of(F, j)
        assert len(L) == d
        keep = np.setdiff1d(np.arange(n), L)
        N = sla.null_space(Ad[keep])
        assert N.shape[1] == d
        b = Ad[j]
        vals = np.abs(grid @ (N.T @ b))  # |b (N c)| for unit c
        best = int(np.argmax(vals))
        assert F.flags[j] & oracle.NULL_CHOICE and F.flags[j] & oracle.RANK_DEFICIENT
        assert not F.flags[j] & oracle.GAP_DEGENERATE
        vjj = v[list(L).index(j)]
        assert abs(vjj.imag) <= 1e-14 * abs(vjj) and vjj.real > 0
        # no grid point is better; the grid's best is within its resolution
        assert vjj.real >= vals[best] - 1e-12
        assert vjj.real <= vals[best] * (1 + hres ** 2) + 1e-12
        assert sin_angle(w, N @ grid[best]) <= 2 * hres
        # w is in the null space: the residual vanishes
        assert F.r[j] <= 1e-12 * np.linalg.norm(Ad)
        # the plain bottom singular vector would generally give less
        assert abs(np.linalg.norm(w) - 1) < 1e-13


def test_null_dimension_one_keeps_the_singular_vector():
    """A one-dimensional null space determines w: no choice is made."""
    n = 7
    rng = np.random.default_rng(5)
    Ad = rng.standard_normal((n, n)) + 3 * np.eye(n)
    A = _csc(Ad)
    full = _pattern([list(range(n))] * n, n)
    F = oracle.factor(A, full, "unit_w", "diag")
    for j in range(n):
        _, w = w_of(F, j)
        N = sla.null_space(np.delete(Ad, j, axis=0))
        assert N.shape[1] == 1
        assert sin_angle(w, N[:, 0]) < 1e-12
        assert F.flags[j] & oracle.RANK_DEFICIENT and not F.flags[j] & oracle.NULL_CHOICE


def test_null_choice_falls_back_when_the_row_is_orthogonal():
    """Row j a combination of the kept rows: P_N b^* = 0, every w in N gives
    v_jj = 0, so the plain bottom singular vector stays (flag SMALL_DIAG)."""
    n = 7
    rng = np.random.default_rng(9)
    Ad = rng.standard_normal((n, n)) + 3 * np.eye(n)
    j = 2
    L = [j, 5]
    keep = np.setdiff1d(np.arange(n), L)
    Ad[j] = rng.standard_normal(keep.size) @ Ad[keep]
    A = _csc(Ad)
    full = _pattern([list(range(n))] * n, n)
    Vexp = _pattern([L if c == j else [c] for c in range(n)], n)
    F = oracle.factor(A, full, "unit_w", "explicit", Vexp=Vexp)
    assert F.flags[j] & oracle.RANK_DEFICIENT
    assert not F.flags[j] & oracle.NULL_CHOICE
    assert F.flags[j] & oracle.SMALL_DIAG
    _, w = w_of(F, j)
    N = sla.null_space(Ad[keep])
    assert N.shape[1] == 2
    assert np.linalg.norm(N.T @ w) > 1 - 1e-12  # still in the null space


# ---------------------------------------------------------------------------
# Rank and gap flags against NumPy's QR and SVD on matrices with nearly
# dependent columns (some below, some above the thresholds).
# ---------------------------------------------------------------------------
def _near_dependent(seed, cplx, eps):
    n = 16
    A = synth.random_small(n, 3, seed, complex_=cplx, diag_shift=2.0)
    Ad = dense(A)
    rng = np.random.default_rng(seed)
    for c in (3, 9):
        pat = (Ad[:, c - 1] != 0)
        Ad[:, c] = np.where(pat, Ad[:, c - 1] * (1 + eps * rng.standard_normal(n)), 0)
        Ad[:, c] += np.where(np.arange(n) == c, 1.0, 0.0) * (Ad[c, c] == 0)
    return _csc(Ad), Ad


@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("eps", [1e-9, 1e-6, 1e-3])
def test_rank_flags_match_numpy(cplx, eps):
    A, Ad = _near_dependent(3 + int(eps < 1e-7), cplx, eps)
    J = oracle.pattern_A2(A)
    seen = {0: 0, 1: 0}
    for mode in ("unit_v", "unit_w"):
        F = oracle.factor(A, J, mode, "topk_lower", 3)
        for j in range(A.n):
            if F.flags[j] & oracle.RANK_EDGE:
                continue
            R, B = _block(Ad, J, j)
            m, k = B.shape
            if mode == "unit_v":
                if k > m:
                    want = True
                else:
                    Rf = np.linalg.qr(B, mode="r")
                    dmin = np.min(np.abs(np.diag(Rf))) ** 2
                    want = dmin <= 1e-14 * np.max(np.sum(np.abs(B) ** 2, axis=0))
            else:
                L, _ = v_of(F, j)
                rows = np.setdiff1d(np.arange(m), np.searchsorted(R, L))
                Ah = B[rows]
                s = np.zeros(k)
                sv = np.linalg.svd(Ah, compute_uv=False)
                s[:sv.size] = sv
                want = Ah.shape[0] < k or s.min() ** 2 <= 1e-14 * np.sum(np.abs(Ah) ** 2)
            got = bool(F.flags[j] & oracle.RANK_DEFICIENT)
            assert got == want, (mode, j)
            seen[int(got)] += 1
    if eps == 1e-9:
        assert seen[1] > 0  # the construction does reach the flag
    assert seen[0] > 0


@pytest.mark.parametrize("cplx", [False, True])
def test_gap_flags_match_numpy(cplx):
    A = synth.random_small(18, 3, 31, complex_=cplx, diag_shift=1.0)
    Ad = dense(A)
    J = oracle.pattern_A2(A)
    for mode in ("unit_v", "unit_w"):
        F = oracle.factor(A, J, mode, "topk_upper", 4)
        for j in range(A.n):
            if F.flags[j] & (oracle.RANK_EDGE | oracle.RANK_DEFICIENT):
                continue
            R, B = _block(Ad, J, j)
            L, _ = v_of(F, j)
            loc = np.searchsorted(R, L)
            if mode == "unit_v":
                Q, _ = np.linalg.qr(B)
                s = np.linalg.svd(Q[loc], compute_uv=False)
                gap = (s[0] ** 2 - s[1] ** 2) / s[0] ** 2 if len(L) >= 2 else 1.0
            else:
                s = np.linalg.svd(np.delete(B, loc, axis=0), compute_uv=False)
                gap = (s[-2] ** 2 - s[-1] ** 2) / s[0] ** 2 if B.shape[1] >= 2 else 1.0
            assert abs(F.gap[j] - gap) <= 1e-10 * max(1.0, gap), (mode, j)
            assert bool(F.flags[j] & oracle.GAP_DEGENERATE) == (gap < 1e-6), (mode, j)


def test_gap_flags_on_degenerate_constructions():
    # unit v, full pattern, |L| = 2: every singular value of M_j is 1
    n = 6
    rng = np.random.default_rng(2)
    Ad = rng.standard_normal((n, n)) + 3 * np.eye(n)
    A = _csc(Ad)
    full = _pattern([list(range(n))] * n, n)
    Vexp = _pattern([sorted({j, (j + 1) % n}) for j in range(n)], n)
    F = oracle.factor(A, full, "unit_v", "explicit", Vexp=Vexp)
    assert np.all(F.flags & oracle.GAP_DEGENERATE)
    # unit w: Ahat = [[1,0],[0,1],[2,0],[0,2]] has sigma_1 = sigma_2 = sqrt(5)
    Ad = np.eye(6) * 4.0
    Ad[:, 0] = [1, 1, 0, 2, 0, 0]
    Ad[:, 1] = [1, 0, 1, 0, 2, 0]
    A = _csc(Ad)
    Jl = [[0, 1]] + [[c] for c in range(1, 6)]
    F = oracle.factor(A, _pattern(Jl, 6), "unit_w", "diag")
    assert F.flags[0] & oracle.GAP_DEGENERATE
    assert not F.flags[0] & oracle.RANK_DEFICIENT
    assert abs(F.r[0] - np.sqrt(5.0)) < 1e-13


# ---------------------------------------------------------------------------
# Phase rule, fallback branch: the diagonal entry is absent or negligible,
# so the entry of largest modulus is made real positive, the lowest row on
# ties.  Expected values from NumPy's QR + SVD of M_j (eq. 2.3).
# ---------------------------------------------------------------------------
def _unit_v_numpy(Ad, J, j, Lrows):
    R, B = _block(Ad, J, j)
    Q, _ = np.linalg.qr(B)
    X = Q[np.searchsorted(R, Lrows)]          # l x k: M_j^*
    U, s, _ = np.linalg.svd(X)
    return U[:, 0]


def _expected_phase(v, rows, j):
    v = np.asarray(v)
    if j in list(rows):
        d = v[list(rows).index(j)]
        if abs(d) >= 1e-8 * np.linalg.norm(v):
            return v * (np.conj(d) / abs(d))
    a = np.abs(v)
    piv = min(np.flatnonzero(a == a.max()), key=lambda t: rows[t])
    return v * (np.conj(v[piv]) / abs(v[piv]))


@pytest.mark.parametrize("cplx,fac", [(False, -1.0), (False, -2.0), (True, -2.0)])
def test_phase_fallback_without_the_diagonal(cplx, fac):
    """Explicit V rows {r1, r2} without j, and row r2 of B = A(R_j, J_j) fac
    times row r1: the rows of Q are too, so v is (1, fac)/||(1, fac)|| up to
    phase.  fac = -2: the entry at r2 is the largest and is made real
    positive.  fac = -1 (real): a tie of moduli, which the lowest row
    decides (v_r1 > 0).  A complex tie is left out: there the moduli are
    equal only up to rounding, which then decides."""
    n = 8
    rng = np.random.default_rng(4)
    Ad = 3.0 * np.eye(n, dtype=complex if cplx else float)
    j, r1, r2, Jj = 1, 3, 6, [0, 2, 4]
    row = rng.standard_normal(3) + (1j * rng.standard_normal(3) if cplx else 0)
    Ad[r1, Jj] = row
    Ad[r2, Jj] = fac * row
    Ad[j, 0] = 0.5  # row j in the shadow of J_j, outside the V pattern
    A = _csc(Ad)
    J = _pattern([Jj if c == j else [c] for c in range(n)], n)
    Vexp = _pattern([[r1, r2] if c == j else [c] for c in range(n)], n)
    F = oracle.factor(A, J, "unit_v", "explicit", Vexp=Vexp)
    L, v = v_of(F, j)
    assert list(L) == [r1, r2]
    assert F.flags[j] & oracle.SMALL_DIAG
    want = _expected_phase(_unit_v_numpy(Ad, J, j, L), L, j)
    assert np.allclose(v, want, atol=1e-12)
    s = np.hypot(1.0, fac)
    if fac == -1.0:
        assert abs(v[0] - 1 / s) < 1e-12 and abs(v[1] + 1 / s) < 1e-12
    else:
        assert abs(v[0] + 1 / s) < 1e-12 and abs(v[1] - 2 / s) < 1e-12


def test_phase_fallback_with_a_negligible_diagonal():
    """j in L_j but |v_jj| < 1e-8 ||v_j||: the largest entry decides."""
    n = 8
    rng = np.random.default_rng(6)
    Ad = 3.0 * np.eye(n)
    j, Jj = 2, [0, 3, 7]
    Ad[:, Jj] += rng.standard_normal((n, 3)) * (rng.random((n, 3)) < 0.6)
    Ad[j, Jj] = [1e-13, 0.0, 0.0]
    A = _csc(Ad)
    J = _pattern([Jj if c == j else [c] for c in range(n)], n)
    Vexp = _pattern([[j, 4, 6] if c == j else [c] for c in range(n)], n)
    F = oracle.factor(A, J, "unit_v", "explicit", Vexp=Vexp)
    L, v = v_of(F, j)
    assert list(L) == [j, 4, 6]
    assert not F.flags[j] & oracle.GAP_DEGENERATE
    assert abs(v[0]) < 1e-8 * np.linalg.norm(v)
    want = _expected_phase(_unit_v_numpy(Ad, J, j, L), L, j)
    assert np.allclose(v, want, atol=1e-12)
    big = int(np.argmax(np.abs(v)))
    assert big != 0 and v[big] > 0
