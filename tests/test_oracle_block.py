"""Pins of the oracle's block diagonal V (Section 5: V the block diagonal
matrices of the splitting A = L + D + U): the pattern of D, the top-k rule
restricted to the block of column j, and the block solve inside W V^{-1}
and BiCGSTAB.

The checks use SciPy / NumPy (dense slicing, LAPACK solves, SciPy's
BiCGSTAB) and brute force over subsets, not the oracle's own routines.
"""
import itertools

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle
import synth
from tests._dense import Aj, dense, smallest_right_sv, spaiq_lstsq, v_of


def _starts(n, sizes):
    st = [0]
    while st[-1] < n:
        st.append(min(n, st[-1] + sizes[(len(st) - 1) % len(sizes)]))
    return np.array(st, dtype=np.int32)


def _block_id(starts, n):
    return np.repeat(np.arange(len(starts) - 1), np.diff(starts))


def test_pattern_of_d_is_the_block_diagonal_part():
    A = synth.random_small(60, 5, 4)
    st = _starts(A.n, [3, 5, 1, 7])
    bid = _block_id(st, A.n)
    Ad = dense(A)
    mask = (Ad != 0) & (bid[:, None] == bid[None, :])
    D = sp.csc_matrix(mask.astype(np.int8))
    D.sort_indices()
    P = oracle.pattern_vblock(A, st)
    assert np.array_equal(P.colptr, D.indptr) and np.array_equal(P.rowidx, D.indices)


@pytest.mark.parametrize("mode", ["unit_v", "unit_w"])
@pytest.mark.parametrize("cplx", [False, True])
def test_topk_block_is_optimal_within_the_block(mode, cplx):
    """The rows chosen are j and the l - 1 rows of j's block in the shadow
    with the largest |(A w0)_i|: they maximise ||(A w0)_L|| over every such
    subset (brute force), w0 the diagonal-V seed from NumPy's least squares
    (unit v) or SVD (unit w)."""
    A = synth.random_small(24, 4, 17, complex_=cplx, diag_shift=1.0)
    Ad = dense(A)
    J = oracle.pattern_A2(A)
    st = _starts(A.n, [6, 4, 8])
    bid = _block_id(st, A.n)
    l = 3
    F = oracle.factor(A, J, mode, "topk_block", vcount=l, vblocks=st)
    checked = 0
    for j in range(A.n):
        A_j = Aj(Ad, J, j)
        R = np.nonzero(np.any(A_j != 0, axis=1))[0]
        w0 = spaiq_lstsq(Ad, J, j) if mode == "unit_v" else smallest_right_sv(Ad, J, j, [j])[0]
        y = A_j @ w0
        adm = [i for i in R if i != j and bid[i] == bid[j]]
        L, _ = v_of(F, j)
        lj = min(l, 1 + len(adm))
        if mode == "unit_w":
            lj = min(lj, max(1, len(R) - A_j.shape[1]))
        assert len(L) == lj and j in L
        assert all(bid[i] == bid[j] for i in L)
        best = max(np.linalg.norm(y[[j, *c]]) for c in itertools.combinations(adm, lj - 1))
        assert np.linalg.norm(y[L]) >= best * (1 - 1e-12)
        checked += lj > 1
    assert checked > A.n // 2


def _vd(F, n):
    return sp.csc_matrix((F.Vval, F.Vri, F.Vcp), shape=(n, n))


@pytest.mark.parametrize("cplx", [False, True])
def test_block_apply_solves_each_block(cplx):
    """W V^{-1} x: V^{-1} x agrees with LAPACK on each dense block and
    satisfies V t = x (SciPy product); blocks of one row reduce to the
    diagonal solve of the triangular path."""
    A = synth.random_small(50, 4, 8, complex_=cplx, diag_shift=2.0)
    J = oracle.pattern_A(A)
    st = _starts(A.n, [5, 2, 9])
    F = oracle.factor(A, J, "unit_v", "explicit", Vexp=oracle.pattern_vblock(A, st))
    rng = np.random.default_rng(0)
    x = rng.standard_normal(A.n) + (1j * rng.standard_normal(A.n) if cplx else 0)
    y = oracle.apply(F, x, "block", st)
    V = _vd(F, A.n)
    W = sp.csc_matrix((F.Wval, F.Jri, F.Jcp), shape=(A.n, A.n))
    Vd = V.toarray()
    t = np.zeros(A.n, dtype=Vd.dtype)
    for b in range(len(st) - 1):
        s = slice(st[b], st[b + 1])
        t[s] = np.linalg.solve(Vd[s, s], x[s])
    assert np.linalg.norm(y - W @ t) <= 1e-12 * np.linalg.norm(W @ t)
    assert np.linalg.norm(V @ t - x) <= 1e-12 * np.linalg.norm(x)
    st1 = np.arange(A.n + 1, dtype=np.int32)
    F1 = oracle.factor(A, J, "unit_v", "diag")
    assert np.array_equal(oracle.apply(F1, x, "block", st1), oracle.apply(F1, x, True))


def test_block_apply_rejects_entries_outside_blocks_and_zero_pivots():
    A = synth.random_small(30, 4, 9, diag_shift=2.0)
    J = oracle.pattern_A(A)
    st = _starts(A.n, [5])
    F = oracle.factor(A, J, "unit_v", "gs_upper")
    with pytest.raises(ValueError):
        oracle.apply(F, np.ones(A.n), "block", st)  # the Gauss-Seidel V crosses blocks
    Fb = oracle.factor(A, J, "unit_v", "explicit", Vexp=oracle.pattern_vblock(A, st))
    Fb.Vval[Fb.Vcp[3]:Fb.Vcp[4]] = 0.0  # column 3 of V zero: its block is singular
    with pytest.raises(ZeroDivisionError):
        oracle.apply(Fb, np.ones(A.n), "block", st)


@pytest.mark.parametrize("mode", ["unit_v", "unit_w"])
def test_bicgstab_with_block_v_matches_scipy(mode):
    """Right-preconditioned BiCGSTAB with M = W V^{-1}, V block diagonal
    (x-lines of the grid as blocks).  SciPy's BiCGSTAB with the same M
    (the block apply, pinned above against LAPACK) takes the same number of
    iterations up to the half-step convention (one); with M from SciPy's
    sparse LU of V, whose pivoting rounds differently, at most two more."""
    A = synth.convdiff(24, 2, 1)
    b = synth.rhs_ones(A)
    st = np.arange(0, A.n + 1, 24, dtype=np.int32)
    J = oracle.pattern_A2(A)
    F = oracle.factor(A, J, mode, "topk_block", vcount=3, vblocks=st)
    x, info = oracle.bicgstab(A, b, F, upper="block", tol=1e-8, maxit=1000, vblocks=st)
    W = sp.csc_matrix((F.Wval, F.Jri, F.Jcp), shape=(A.n, A.n)).tocsr()
    lu = spla.splu(_vd(F, A.n).tocsc())
    assert info.flag == 0
    assert np.linalg.norm(A.to_scipy() @ x - b) <= 1.01e-8 * np.linalg.norm(b)
    for Mf, slack in ((lambda z: oracle.apply(F, z, "block", st), 1),
                      (lambda z: W @ lu.solve(z), 2)):
        M = spla.LinearOperator(A.to_scipy().shape, matvec=Mf)
        its = [0]
        xs, flag = spla.bicgstab(A.to_scipy(), b, M=M, rtol=1e-8, atol=0.0, maxiter=1000,
                                 callback=lambda xk: its.__setitem__(0, its[0] + 1))
        assert flag == 0
        assert abs(its[0] - info.iters) <= slack
