"""Pins of the CPU oracle against things other than itself.

Each test names the passage of the paper it rests on.  None re-runs the
oracle's own routines: they use LAPACK least squares / SVD / inverse through
NumPy, SciPy's sparse products, triangular solve and BiCGSTAB, brute force
over unit vectors and over subsets, closed forms, and special cases with a
known exact answer.
"""
import itertools

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle
import synth
from tests._dense import (Aj, cols_of, dense, sin_angle, smallest_right_sv, spaiq_lstsq,
                          trsv_scipy, v_of, w_of)

SEEDS = [11, 12, 13]


def _small(seed, complex_=False, n=14, per_col=3):
    return synth.random_small(n, per_col, seed, complex_=complex_, diag_shift=2.0)


# ---------------------------------------------------------------------------
# P1: with the diagonal V (V_0 = diagonals) the first basic algorithm is the
# sparse approximate inverse: v_j = e_j and w_j = argmin ||A_j w - e_j||
# (Example 2.1, Example 3.2).
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("seed", SEEDS)
@pytest.mark.parametrize("cplx", [False, True])
def test_p1_spai_special_case(seed, cplx):
    A = _small(seed, cplx)
    Ad = dense(A)
    J = oracle.pattern_A2(A)
    F = oracle.factor(A, J, "unit_v", "diag")
    for j in range(A.n):
        rows, vals = v_of(F, j)
        assert list(rows) == [j]
        assert abs(vals[0] - 1.0) < 1e-14
        _, w = w_of(F, j)
        wref = spaiq_lstsq(Ad, J, j)
        assert np.linalg.norm(w - wref) <= 1e-11 * np.linalg.norm(wref)
        # residual equals the least-squares residual
        e = np.zeros(A.n, dtype=Ad.dtype)
        e[j] = 1
        assert abs(F.r[j] - np.linalg.norm(Aj(Ad, J, j) @ wref - e)) <= 1e-12


# ---------------------------------------------------------------------------
# P2 + P3: the second basic algorithm takes w_j as the right singular vector
# of sigma_min of A_j with the rows L_j removed, v_j = (A w_j) on L_j, and
# then ||A w_j - v_j|| = sigma_min (Section 2.2).
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("seed", SEEDS)
@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("vrule", ["diag", "gs_upper", "gs_lower"])
def test_p2_diafs_smallest_singular_vector(seed, cplx, vrule):
    A = _small(seed, cplx)
    Ad = dense(A)
    J = oracle.pattern_A2(A)
    F = oracle.factor(A, J, "unit_w", vrule)
    for j in range(A.n):
        L, v = v_of(F, j)
        _, w = w_of(F, j)
        wref, s = smallest_right_sv(Ad, J, j, L)
        assert abs(np.linalg.norm(w) - 1) < 1e-13
        if F.flags[j] & (oracle.GAP_DEGENERATE | oracle.RANK_DEFICIENT):
            continue
        assert sin_angle(w, wref) < 1e-10
        Aw = Aj(Ad, J, j) @ w
        assert np.allclose(v, Aw[L], atol=1e-13)
        assert abs(F.r[j] - s[-1]) <= 1e-12 * max(1.0, s[0])
        assert abs(F.rclosed[j] - s[-1]) <= 1e-12 * max(1.0, s[0])


@pytest.mark.parametrize("seed", SEEDS)
@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("vrule", ["gs_upper", "gs_lower"])
def test_p3_diafq_closed_form(seed, cplx, vrule):
    """First basic algorithm: v_j maximises ||M_j v|| over unit v with
    M_j = (rows L_j of an orthonormal basis Q_j of range(A_j))^* (eq. (2.3)),
    w_j solves the least-squares problem (2.4), and the residual squared is
    1 - ||M_j||^2."""
    A = _small(seed, cplx)
    Ad = dense(A)
    J = oracle.pattern_A2(A)
    F = oracle.factor(A, J, "unit_v", vrule)
    for j in range(A.n):
        L, v = v_of(F, j)
        _, w = w_of(F, j)
        A_j = Aj(Ad, J, j)
        Q, _ = np.linalg.qr(A_j)
        M = Q[L, :].conj().T
        U, s, Vh = np.linalg.svd(M)
        assert abs(np.linalg.norm(v) - 1) < 1e-13
        assert abs(F.r[j] ** 2 - (1 - s[0] ** 2)) < 1e-12
        if not F.flags[j] & oracle.GAP_DEGENERATE:
            assert sin_angle(v, Vh[0].conj()) < 1e-10
        vext = np.zeros(A.n, dtype=Ad.dtype)
        vext[L] = v
        wls = np.linalg.lstsq(A_j, vext, rcond=None)[0]
        assert np.linalg.norm(w - wls) <= 1e-10 * max(1.0, np.linalg.norm(wls))
        assert abs(F.r[j] - np.linalg.norm(A_j @ w - vext)) < 1e-12


# ---------------------------------------------------------------------------
# P4: brute force over unit vectors on tiny columns (problem (1.2) with a
# fixed-norm constraint): the oracle must not lose to any grid point.
# ---------------------------------------------------------------------------
def _fib_sphere(npts):
    i = np.arange(npts) + 0.5
    phi = np.arccos(1 - 2 * i / npts)
    th = np.pi * (1 + 5 ** 0.5) * i
    return np.stack([np.cos(th) * np.sin(phi), np.sin(th) * np.sin(phi), np.cos(phi)], axis=1)


def _unit_grid(d):
    """Unit vectors covering the half sphere (sign is free) and the grid's
    worst-case angle to any unit vector."""
    if d == 1:
        return np.array([[1.0]]), 0.0
    if d == 2:
        t = np.linspace(0, np.pi, 20001)
        return np.stack([np.cos(t), np.sin(t)], axis=1), np.pi / 20000
    npts = 200000
    return _fib_sphere(npts), 2.0 * np.sqrt(4 * np.pi / npts)


def test_p4_brute_force_unit_v():
    A = synth.random_small(8, 1, 5, diag_shift=0.5)
    Ad = dense(A)
    J = oracle.pattern_A(A)
    F = oracle.factor(A, J, "unit_v", "gs_upper")
    checked = 0
    for j in range(A.n):
        L, v = v_of(F, j)
        if len(L) < 2 or len(L) > 3:
            continue
        A_j = Aj(Ad, J, j)
        Q, _ = np.linalg.qr(A_j)
        P = np.eye(A.n) - Q @ Q.T
        best = np.inf
        grid, h = _unit_grid(len(L))
        for u in grid:
            vext = np.zeros(A.n)
            vext[L] = u
            best = min(best, np.linalg.norm(P @ vext))
        # never worse than a grid point; better by at most the grid's
        # resolution (the squared objective is quadratic with curvature <= 1)
        assert F.r[j] <= best + 1e-12
        assert F.r[j] ** 2 >= best ** 2 - h ** 2
        checked += 1
    assert checked >= 2


def test_p4_brute_force_unit_w():
    A = synth.random_small(9, 2, 6, diag_shift=0.5)
    Ad = dense(A)
    J = oracle.pattern_A(A)
    F = oracle.factor(A, J, "unit_w", "gs_lower")
    checked = 0
    for j in range(A.n):
        L, v = v_of(F, j)
        k = F.Jcp[j + 1] - F.Jcp[j]
        if k > 3:
            continue
        A_j = Aj(Ad, J, j)
        keep = np.setdiff1d(np.arange(A.n), L)
        best = np.inf
        grid, h = _unit_grid(k)
        for u in grid:
            best = min(best, np.linalg.norm(A_j[keep] @ u))
        smax = np.linalg.norm(A_j[keep], 2)
        assert F.r[j] <= best + 1e-12
        assert F.r[j] ** 2 >= best ** 2 - (h * smax) ** 2
        checked += 1
    assert checked >= 3


# ---------------------------------------------------------------------------
# P5: exact case.  With full W patterns and V_0 = diagonals, W V^{-1} = A^{-1}
# and every residual vanishes (Theorem 2.1: the column scaling is free).
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("mode", ["unit_v", "unit_w"])
@pytest.mark.parametrize("cplx", [False, True])
def test_p5_exact_case_full_pattern(mode, cplx):
    n = 12
    A = synth.random_small(n, n - 1, 21, complex_=cplx, diag_shift=3.0)
    Ad = dense(A)
    full = oracle.Pattern(n, np.arange(0, n * n + 1, n, dtype=np.int32),
                          np.tile(np.arange(n, dtype=np.int32), n))
    F = oracle.factor(A, full, mode, "diag")
    W = F.W_scipy().toarray()
    V = F.V_scipy().toarray()
    assert np.allclose(W @ np.linalg.inv(V), np.linalg.inv(Ad), atol=1e-10)
    assert np.max(F.r) < 1e-12
    x, info = oracle.bicgstab(A, synth.rhs_ones(A), F, upper=False)
    assert info.flag == 0 and info.iters == 1
    assert np.allclose(x, 1.0, atol=1e-10)


def test_p5_exact_case_block_diagonal():
    """Block-diagonal A with J_j = the block of j: each block is inverted exactly."""
    rng = np.random.default_rng(3)
    blocks = [rng.standard_normal((b, b)) + 3 * np.eye(b) for b in (3, 4, 2, 5)]
    Ad = sp.block_diag(blocks).toarray()
    A = synth.CSC.from_scipy(sp.csc_matrix(Ad))
    n = A.n
    cp, ri, off = [0], [], 0
    for b in blocks:
        for _ in range(b.shape[0]):
            ri += list(range(off, off + b.shape[0]))
            cp.append(len(ri))
        off += b.shape[0]
    J = oracle.Pattern(n, np.array(cp, np.int32), np.array(ri, np.int32))
    for mode in ("unit_v", "unit_w"):
        F = oracle.factor(A, J, mode, "diag")
        W = F.W_scipy().toarray()
        V = F.V_scipy().toarray()
        assert np.allclose(W @ np.linalg.inv(V), np.linalg.inv(Ad), atol=1e-11)
        assert np.max(F.r) < 1e-12


# ---------------------------------------------------------------------------
# P6: rows orthogonal (A A^* diagonal) and W pattern = pattern(A^*) give the
# exact factoring A W V^{-1} = I with V diagonal (Example 4.2).
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("cplx", [False, True])
def test_p6_orthogonal_rows(cplx):
    rng = np.random.default_rng(7)
    blocks = []
    for b in (2, 3, 2, 4, 3):
        X = rng.standard_normal((b, b)) + (1j * rng.standard_normal((b, b)) if cplx else 0)
        Q, _ = np.linalg.qr(X)
        blocks.append(Q)
    U = sp.block_diag(blocks).toarray()
    D = np.diag(rng.uniform(0.5, 3.0, U.shape[0]))
    Ad = D @ U
    perm = rng.permutation(U.shape[0])
    Ad = Ad[:, perm]  # still A A^* = D^2
    A = synth.CSC.from_scipy(sp.csc_matrix(Ad))
    AT = synth.CSC.from_scipy(sp.csc_matrix(Ad.conj().T))
    J = oracle.Pattern(A.n, AT.colptr, AT.rowidx)
    for mode in ("unit_v", "unit_w"):
        F = oracle.factor(A, J, mode, "diag")
        W = F.W_scipy().toarray()
        V = F.V_scipy().toarray()
        assert np.allclose(Ad @ W @ np.linalg.inv(V), np.eye(A.n), atol=1e-12)
        assert np.max(F.r) < 1e-13


# ---------------------------------------------------------------------------
# P7: the V pattern chosen by top-k over |A w0| maximises ||(A w0)_L|| over
# all admissible L containing j with |L| = l, and therefore minimises
# min_v ||A w0 - v|| for that w0 in both norm modes (Section 3.1).
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("mode", ["unit_v", "unit_w"])
@pytest.mark.parametrize("tri", ["lower", "upper"])
@pytest.mark.parametrize("cplx", [False, True])
def test_p7_topk_is_optimal(mode, tri, cplx):
    A = synth.random_small(16, 3, 31, complex_=cplx, diag_shift=1.0)
    Ad = dense(A)
    J = oracle.pattern_A(A)
    l = 3
    F = oracle.factor(A, J, mode, "topk_" + tri, vcount=l)
    for j in range(A.n):
        A_j = Aj(Ad, J, j)
        R = np.nonzero(np.any(A_j != 0, axis=1))[0]
        if mode == "unit_v":
            w0 = spaiq_lstsq(Ad, J, j)
        else:
            w0, _ = smallest_right_sv(Ad, J, j, [j])
        y = A_j @ w0
        adm = [i for i in R if (i > j if tri == "lower" else i < j)]
        L, _ = v_of(F, j)
        lj = min(l, 1 + len(adm))
        if mode == "unit_w":
            lj = min(lj, max(1, len(R) - A_j.shape[1]))
        assert len(L) == lj and j in L
        best = max(np.linalg.norm(y[[j, *c]]) for c in itertools.combinations(adm, lj - 1))
        assert np.linalg.norm(y[L]) >= best * (1 - 1e-12)

        # the same subset minimises the fixed-w objective directly
        def obj(Ls):
            if mode == "unit_w":
                return np.linalg.norm(y) ** 2 - np.linalg.norm(y[Ls]) ** 2
            return np.linalg.norm(y) ** 2 + 1 - 2 * np.linalg.norm(y[Ls])
        best_obj = min(obj([j, *c]) for c in itertools.combinations(adm, lj - 1))
        assert obj(list(L)) <= best_obj + 1e-12


def test_p7_tie_band_prefers_lower_rows():
    """Exact ties in the scores are resolved by ascending row index."""
    # Swapping rows 1<->2, 4<->5 and columns 1<->2 maps A to itself, so for
    # column 0 the seed gives |(A w0)_1| = |(A w0)_2| and
    # |(A w0)_4| = |(A w0)_5| in exact arithmetic.
    n = 6
    Ad = 4 * np.eye(n)
    for (i, j, a) in [(1, 0, -1), (2, 0, -1), (0, 1, -1), (0, 2, -1), (3, 1, -.5), (3, 2, -.5),
                      (4, 1, -2), (5, 2, -2)]:
        Ad[i, j] = a
    A = synth.CSC.from_scipy(sp.csc_matrix(Ad))
    J = oracle.Pattern(n, A.colptr, A.rowidx)
    y = np.abs(Aj(Ad, J, 0) @ spaiq_lstsq(Ad, J, 0))
    assert abs(y[1] - y[2]) <= 1e-13 * y[1] and abs(y[4] - y[5]) <= 1e-13 * y[4]
    order = sorted(range(1, n), key=lambda i: -y[i])
    first_pair = sorted(order[:2])
    assert abs(y[first_pair[0]] - y[first_pair[1]]) <= 1e-13 * y[first_pair[0]]
    F = oracle.factor(A, J, "unit_v", "topk_lower", vcount=2)
    L, _ = v_of(F, 0)
    assert list(L) == [0, first_pair[0]]
    F = oracle.factor(A, J, "unit_v", "topk_lower", vcount=3)
    L, _ = v_of(F, 0)
    assert list(L) == [0] + first_pair


# ---------------------------------------------------------------------------
# P8: Theorem 2.1 -- any nonzero column scaling D leaves W V^{-1} unchanged.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("cplx", [False, True])
def test_p8_scaling_invariance_of_apply(cplx):
    A = synth.convdiff(8, 2, 4) if not cplx else synth.helmholtz(8, 10.0, 0.5)
    J = oracle.pattern_A2(A)
    F = oracle.factor(A, J, "unit_v", "topk_upper", vcount=3)
    rng = np.random.default_rng(1)
    d = rng.uniform(0.3, 3, A.n) * (np.exp(1j * rng.uniform(0, 6.28, A.n)) if cplx else
                                    rng.choice([-1, 1], A.n))
    F2 = oracle.Factors(**{**F.__dict__})
    F2.Wval = F.Wval * np.repeat(d, np.diff(F.Jcp))
    F2.Vval = F.Vval * np.repeat(d, np.diff(F.Vcp))
    x = rng.standard_normal(A.n) + (1j * rng.standard_normal(A.n) if cplx else 0)
    y1 = oracle.apply(F, x, upper=True)
    y2 = oracle.apply(F2, x, upper=True)
    assert np.allclose(y1, y2, rtol=1e-12, atol=1e-12)
    # and the apply itself against SciPy's triangular solve and product
    t = trsv_scipy(F.V_scipy(), x, upper=True)
    assert np.allclose(y1, F.W_scipy() @ t, rtol=1e-11, atol=1e-12)


# ---------------------------------------------------------------------------
# P9: bound (3.1): ||AWV^{-1}-I||/||V^{-1}|| <= ||AW-V|| <= ||AWV^{-1}-I|| ||V||
# on the 32 x 32 convection-diffusion problem, Frobenius/2-norms.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("mode", ["unit_v", "unit_w"])
def test_p9_bound_3_1(mode):
    A = synth.convdiff(32, 2, 1)
    Ad = dense(A)
    J = oracle.pattern_A(A)
    F = oracle.factor(A, J, mode, "gs_upper")
    W = F.W_scipy().toarray()
    V = F.V_scipy().toarray()
    nrm_direct = np.linalg.norm(Ad @ W - V, "fro")
    nrm = np.sqrt(np.sum(F.r ** 2))
    assert abs(nrm - nrm_direct) <= 1e-10 * nrm_direct
    E = Ad @ W @ np.linalg.inv(V) - np.eye(A.n)
    e = np.linalg.norm(E, "fro")
    assert e / np.linalg.norm(np.linalg.inv(V), 2) <= nrm * (1 + 1e-10)
    assert nrm <= e * np.linalg.norm(V, 2) * (1 + 1e-10)


# ---------------------------------------------------------------------------
# P10: ||M||_F / sqrt(min(k, l)) <= ||M||_2 <= ||M||_F for the matrix of
# Section 3.1 (stated there with max{k,l}; min is the sharper valid form).
# ---------------------------------------------------------------------------
def test_p10_norm_bounds_for_M():
    A = synth.random_small(15, 3, 41, diag_shift=1.0)
    Ad = dense(A)
    J = oracle.pattern_A2(A)
    F = oracle.factor(A, J, "unit_v", "gs_lower")
    for j in range(A.n):
        L, _ = v_of(F, j)
        Q, _ = np.linalg.qr(Aj(Ad, J, j))
        M = Q[L, :].conj().T
        s1 = np.sqrt(max(0.0, 1 - F.r[j] ** 2))  # ||M||_2 from the oracle's residual
        fro = np.linalg.norm(M, "fro")
        assert fro / np.sqrt(min(M.shape)) <= s1 + 1e-10
        assert s1 <= fro + 1e-10


# ---------------------------------------------------------------------------
# P11: BiCGSTAB iteration count against SciPy's (same Templates algorithm,
# right-preconditioned form, independent code).
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("mode", ["unit_v", "unit_w"])
def test_p11_bicgstab_matches_scipy(mode):
    A = synth.convdiff(32, 2, 1)
    b = synth.rhs_ones(A)
    J = oracle.pattern_A(A)
    F = oracle.factor(A, J, mode, "gs_upper")
    x, info = oracle.bicgstab(A, b, F, upper=True, tol=1e-8, maxit=1000)
    W = F.W_scipy().tocsr()
    Vc = F.V_scipy().tocsr()
    M = spla.LinearOperator(A.to_scipy().shape,
                            matvec=lambda z: W @ spla.spsolve_triangular(Vc, z, lower=False))
    its = [0]
    xs, flag = spla.bicgstab(A.to_scipy(), b, M=M, rtol=1e-8, atol=0.0, maxiter=1000,
                             callback=lambda xk: its.__setitem__(0, its[0] + 1))
    assert flag == 0 and info.flag == 0
    assert abs(its[0] - info.iters) <= 1
    assert np.linalg.norm(A.to_scipy() @ x - b) <= 1.01e-8 * np.linalg.norm(b)
    assert np.allclose(x, 1.0, atol=1e-5)


def test_bicgstab_breakdown_and_maxit():
    # skew-symmetric A: <r, A r> = 0 so the first step breaks down
    n = 10
    Ad = np.zeros((n, n))
    for i in range(n - 1):
        Ad[i, i + 1] = 1.0
        Ad[i + 1, i] = -1.0
    A = synth.CSC.from_scipy(sp.csc_matrix(Ad))
    _, info = oracle.bicgstab(A, np.ones(n))
    assert info.flag == 2 and info.iters == 1
    A = synth.convdiff(16, 2, 2)
    _, info = oracle.bicgstab(A, synth.rhs_ones(A), maxit=1)
    assert info.flag == 1 and info.iters == 1


# ---------------------------------------------------------------------------
# Patterns.
# ---------------------------------------------------------------------------
def test_pattern_a2_matches_scipy_product():
    A = synth.random_small(40, 3, 8)
    P = A.to_scipy().copy()
    P.data[:] = 1.0
    ref = (P @ P).tocsc()
    ref.sort_indices()
    J = oracle.pattern_A2(A)
    assert np.array_equal(J.colptr, ref.indptr) and np.array_equal(J.rowidx, ref.indices)
    A = synth.convdiff(16, 3, 2)
    J = oracle.pattern_A2(A)
    k = np.diff(J.colptr)
    assert k.max() == 25 and k.min() == 10


@pytest.mark.parametrize("cplx", [False, True])
def test_pattern_1hop_topk_brute_force(cplx):
    A = synth.random_small(60, 4, 9, complex_=cplx)
    Ad = np.abs(dense(A))
    S = Ad @ Ad
    J = oracle.pattern_1hop(A, 3)
    for j in range(A.n):
        base = set(np.nonzero(Ad[:, j])[0])
        cand = [i for i in np.nonzero(S[:, j])[0] if i not in base]
        cand.sort(key=lambda i: (-S[i, j], i))
        want = sorted(base | set(cand[:3]))
        assert list(cols_of(J, j)) == want


def test_gs_pattern_is_triangle_of_A():
    """Definition 4.1: Gauss-Seidel structure = diagonal + strictly upper part."""
    A = synth.convdiff(10, 2, 3)
    J = oracle.pattern_A(A)
    F = oracle.factor(A, J, "unit_v", "gs_upper")
    T = sp.triu(A.to_scipy()).tocsc()
    T.sort_indices()
    assert np.array_equal(F.Vcp, T.indptr) and np.array_equal(F.Vri, T.indices)


def test_equal_column_structures_give_equal_v_columns():
    """Two columns with the same W and V patterns produce the same V column
    (Section 3.1), hence a singular V."""
    A = synth.random_small(10, 3, 12, diag_shift=2.0)
    n = A.n
    Jl = [list(cols_of(A, j)) for j in range(n)]
    Jl[4] = sorted(set(Jl[3]) | {4})
    Jl[3] = list(Jl[4])
    J = oracle.Pattern(n, np.cumsum([0] + [len(x) for x in Jl]).astype(np.int32),
                       np.array(sum(Jl, []), np.int32))
    Vl = [[j] for j in range(n)]
    Vl[3] = [3, 4]
    Vl[4] = [3, 4]
    Vp = oracle.Pattern(n, np.cumsum([0] + [len(x) for x in Vl]).astype(np.int32),
                        np.array(sum(Vl, []), np.int32))
    F = oracle.factor(A, J, "unit_v", "explicit", Vexp=Vp)
    _, v3 = v_of(F, 3)
    _, v4 = v_of(F, 4)
    assert sin_angle(v3, v4) < 1e-12


def test_phase_rule_and_flags():
    A = synth.helmholtz(16, 20.0, 0.5)
    J = oracle.pattern_A2(A)
    F = oracle.factor(A, J, "unit_w", "topk_upper", vcount=7)
    for j in range(A.n):
        L, v = v_of(F, j)
        d = v[list(L).index(j)]
        if abs(d) >= 1e-8 * np.linalg.norm(v):
            assert abs(d.imag) < 1e-14 * abs(d) and d.real > 0
    # identical columns make B_j rank deficient: flagged
    Ad = dense(synth.random_small(10, 3, 2, diag_shift=2.0))
    Ad[:, 5] = Ad[:, 4]
    Ad[5, 5] += 0.0
    A2 = synth.CSC.from_scipy(sp.csc_matrix(Ad))
    Jl = [sorted(set(cols_of(A2, j)) | {4, 5}) if j in (4, 5) else list(cols_of(A2, j))
          for j in range(A2.n)]
    J2 = oracle.Pattern(A2.n, np.cumsum([0] + [len(x) for x in Jl]).astype(np.int32),
                        np.array(sum(Jl, []), np.int32))
    F2 = oracle.factor(A2, J2, "unit_v", "diag")
    assert F2.flags[4] & oracle.RANK_DEFICIENT
