"""Pins of the oracle's Algorithm 2 W pattern (Section 4): column j of W has
the pattern of A^* v_j for a generic v_j in V_0."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import synth
from tests._dense import Aj, dense, v_of, w_of


def _v0_dense(A, v0, rng):
    """A random matrix with the pattern of V_0 (nonzero values w.p. one)."""
    Ad = dense(A)
    n = A.n
    mask = np.eye(n, dtype=bool)
    nz = Ad != 0
    if v0 == "gs_upper":
        mask |= np.triu(nz, 1)
    elif v0 == "gs_lower":
        mask |= np.tril(nz, -1)
    return np.where(mask, rng.standard_normal((n, n)) + 0.5, 0.0)


@pytest.mark.parametrize("v0", ["diag", "gs_upper", "gs_lower"])
@pytest.mark.parametrize("cplx", [False, True])
def test_alg2_is_the_pattern_of_a_star_v(v0, cplx):
    """The algorithm's definition with random values: the nonzero pattern of
    A^* V for a random V with V_0's pattern (dense NumPy product)."""
    A = synth.random_small(80, 3, 2, complex_=cplx)
    P = oracle.pattern_alg2(A, v0)
    W = dense(A).conj().T @ _v0_dense(A, v0, np.random.default_rng(1))
    for j in range(A.n):
        want = np.nonzero(np.abs(W[:, j]) > 0)[0]
        got = P.rowidx[P.colptr[j]:P.colptr[j + 1]]
        assert np.array_equal(got, want), j


def test_alg2_diagonal_v0_gives_pattern_of_a_star():
    """With V_0 the diagonal matrices the pattern of W is that of A^*."""
    A = synth.convdiff(8, 3, 4)
    P = oracle.pattern_alg2(A, "diag")
    At = A.to_scipy().T.tocsc()
    At.sort_indices()
    assert np.array_equal(P.colptr, At.indptr)
    assert np.array_equal(P.rowidx, At.indices)


def test_alg2_is_monotone_in_v0():
    """V_0 within V_0' gives W within W' (the remark after Example 4.2)."""
    A = synth.random_small(120, 4, 7)
    Pd = oracle.pattern_alg2(A, "diag")
    for v0 in ("gs_upper", "gs_lower"):
        Pg = oracle.pattern_alg2(A, v0)
        for j in range(A.n):
            a = set(Pd.rowidx[Pd.colptr[j]:Pd.colptr[j + 1]])
            b = set(Pg.rowidx[Pg.colptr[j]:Pg.colptr[j + 1]])
            assert a <= b


def test_alg2_orthogonal_rows_give_the_exact_inverse():
    """Example 4.1: with V_0 diagonal and A with orthogonal rows, W = the
    pattern of A^* holds A^{-1} up to column scaling: the diagonal V and
    AW = V exactly."""
    rng = np.random.default_rng(3)
    n = 60
    perm = rng.permutation(n)
    d = rng.uniform(1.0, 2.0, n)
    M = sp.csc_matrix((d, (np.arange(n), perm)), shape=(n, n))  # rows orthogonal
    A = synth.CSC(n=n, colptr=M.indptr.astype(np.int32), rowidx=M.indices.astype(np.int32),
                  val=M.data.astype(np.float64))
    J = oracle.pattern_alg2(A, "diag")
    F = oracle.factor(A, J, "unit_v", "diag")
    assert np.max(F.r) <= 1e-14
