"""Pins of the oracle's Algorithm 1 W pattern (Section 4, sparsified powers
with V_0 the diagonal matrices): S = D^{-1}(A - D), columns of S dropped by
(tau_i, p_i), then per column j k steps t <- S t dropped by (tau_l, p_l), the
pattern of w_j the union of e_j and every kept t.

The checks use SciPy's structural matrix powers, closed forms for one step,
and an independent dense NumPy re-implementation (whole-vector products,
boolean structure masks, argsort-based selection) in place of the oracle's
per-row sparse accumulation.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import synth
from tests._dense import dense


def _cols(P):
    return [list(P.rowidx[P.colptr[j]:P.colptr[j + 1]]) for j in range(P.n)]


def _structural_power(A, k):
    """Pattern of (I + |A - D|)^k: every row reachable from j in at most k
    steps of the off-diagonal graph (positive values: no cancellation)."""
    M = A.to_scipy().tocsc()
    B = (abs(M) > 0).astype(np.int64)
    B.setdiag(0)
    B.eliminate_zeros()
    I = sp.identity(A.n, dtype=np.int64, format="csc")
    R = I.copy()
    for _ in range(k):
        R = ((I + B) @ R).tocsc()
        R.data[:] = 1
    R.sort_indices()
    return [sorted(R.indices[R.indptr[j]:R.indptr[j + 1]]) for j in range(A.n)]


def _keep(vals, mask, tau, p, j):
    """Dense selection: within `mask`, the entries other than j with
    |v| >= tau max|v| (tau > 0), then the p largest by |v| (ties to the lower
    index); entry j (None: no such entry) is kept whenever it is in the
    mask."""
    idx = np.nonzero(mask)[0]
    if idx.size == 0:
        return mask.copy()
    a = np.abs(vals[idx])
    cand = idx if j is None else idx[idx != j]
    if tau > 0:
        cand = cand[np.abs(vals[cand]) >= tau * a.max()]
    if p > 0 and cand.size > p:
        order = np.lexsort((cand, -np.abs(vals[cand])))
        cand = cand[order[:p]]
    out = np.zeros_like(mask)
    out[cand] = True
    if j is not None and mask[j]:
        out[j] = True
    return out


def _dense_alg1(A, k, tau_i, p_i, tau_l, p_l):
    Ad = dense(A)
    n = A.n
    d = np.diag(Ad).copy()
    S = (Ad - np.diag(d)) / d[:, None]  # row i scaled by 1 / a_ii
    Smask = (Ad != 0) & ~np.eye(n, dtype=bool)
    for c in range(n):
        Smask[:, c] = _keep(S[:, c], Smask[:, c], tau_i, p_i, None)
    S = np.where(Smask, S, 0.0)
    Si = Smask.astype(np.int64)
    out = []
    for j in range(n):
        t = np.zeros(n)
        t[j] = 1.0
        tm = np.zeros(n, dtype=bool)
        tm[j] = True
        s = tm.copy()
        for _ in range(k):
            t = S @ t
            tm = (Si @ tm.astype(np.int64)) > 0
            tm = _keep(t, tm, tau_l, p_l, j)
            t = np.where(tm, t, 0.0)
            s |= tm
        out.append(list(np.nonzero(s)[0]))
    return out


def test_one_step_without_dropping_is_the_pattern_of_a():
    A = synth.random_small(90, 4, 11)
    P = oracle.pattern_sparsified_powers(A, k=1, tau_i=0.0)
    Q = oracle.pattern_A(A)
    assert np.array_equal(P.colptr, Q.colptr) and np.array_equal(P.rowidx, Q.rowidx)


@pytest.mark.parametrize("k", [2, 3, 4])
def test_no_dropping_is_the_structural_truncated_series(k):
    """Without dropping the pattern of I + S + ... + S^k is that of
    (I + |A - D|)^k (for k = 2 also that of A^2, with the diagonal full)."""
    A = synth.random_small(70, 3, 12 + k)
    P = oracle.pattern_sparsified_powers(A, k=k, tau_i=0.0)
    assert _cols(P) == _structural_power(A, k)
    if k == 2:
        Q = oracle.pattern_A2(A)
        assert _cols(P) == _cols(Q)


@pytest.mark.parametrize("tau,p", [(0.3, 0), (0.0, 2), (0.5, 1)])
def test_one_step_closed_form_of_initial_dropping(tau, p):
    """k = 1: column j is {j} and the off-diagonal rows i of A(:, j) whose
    |a_ij / a_ii| pass the tolerance relative to the column's largest, at
    most p of them (the largest).  Diagonals differ from row to row, so
    scaling by a_jj instead of a_ii fails this."""
    A = synth.random_small(80, 5, 21)
    Ad = dense(A)
    P = oracle.pattern_sparsified_powers(A, k=1, tau_i=tau, p_i=p)
    for j, got in enumerate(_cols(P)):
        rows = [i for i in range(A.n) if i != j and Ad[i, j] != 0]
        m = np.array([abs(Ad[i, j] / Ad[i, i]) for i in rows])
        keep = [r for r, x in zip(rows, m) if tau == 0 or x >= tau * m.max()]
        if p and len(keep) > p:
            mk = {r: x for r, x in zip(rows, m)}
            keep = sorted(keep, key=lambda r: (-mk[r], r))[:p]
        assert got == sorted(keep + [j]), j


def test_count_ties_go_to_the_lower_row():
    """Laplacian (no convection): every off-diagonal of S is -1/4, so p_i = 2
    keeps the two lowest rows of each column."""
    A = synth.convdiff(6, 2, 0, beta_max=0.0)
    Ad = dense(A)
    P = oracle.pattern_sparsified_powers(A, k=1, tau_i=0.0, p_i=2)
    for j, got in enumerate(_cols(P)):
        rows = [i for i in range(A.n) if i != j and Ad[i, j] != 0]
        assert got == sorted(rows[:2] + [j]), j


@pytest.mark.parametrize("k,tau_i,p_i,tau_l,p_l", [
    (2, 0.1, 0, 0.0, 0),
    (3, 0.1, 0, 0.0, 0),
    (3, 0.0, 0, 0.2, 0),
    (3, 0.05, 3, 0.1, 4),
    (4, 0.0, 2, 0.0, 3),
    (3, 0.0, 0, 0.99, 1),
])
def test_matches_dense_reimplementation(k, tau_i, p_i, tau_l, p_l):
    A = synth.random_small(60, 4, 31 + k)
    P = oracle.pattern_sparsified_powers(A, k=k, tau_i=tau_i, p_i=p_i, tau_l=tau_l, p_l=p_l)
    assert _cols(P) == _dense_alg1(A, k, tau_i, p_i, tau_l, p_l)


def test_diagonal_of_t_is_never_dropped():
    """With tau_l = 0.99 and p_l = 1 each t keeps one off-diagonal entry;
    whenever row j reappears in t (a path j -> i -> j) it is kept, so its
    successors reach s_j.  The dense version agrees, and keeping j matters
    for some columns (dropping it there gives a different pattern)."""
    A = synth.random_small(60, 4, 5)
    P = _cols(oracle.pattern_sparsified_powers(A, k=3, tau_i=0.0, tau_l=0.99, p_l=1))
    assert P == _dense_alg1(A, 3, 0.0, 0, 0.99, 1)
    Ad = dense(A)
    d = np.diag(Ad)
    S = np.where(np.eye(A.n, dtype=bool), 0.0, Ad / d[:, None])
    differs = 0
    for j in range(A.n):
        # the same expansion with row j subject to dropping like the others
        t = np.zeros(A.n)
        t[j] = 1.0
        s = {j}
        for _ in range(3):
            t = S @ t
            nz = np.nonzero(t)[0]
            a = np.abs(t[nz])
            keep = nz[a >= 0.99 * a.max()]
            keep = keep[np.lexsort((keep, -np.abs(t[keep])))][:1]
            t = np.where(np.isin(np.arange(A.n), keep), t, 0.0)
            s |= set(keep.tolist())
        differs += sorted(s) != P[j]
    assert differs > 0


def test_zero_diagonal_is_rejected():
    A = synth.random_small(20, 3, 1)
    dpos = [q for q in range(A.colptr[4], A.colptr[5]) if A.rowidx[q] == 4][0]
    A.val[dpos] = 0.0
    with pytest.raises(ValueError):
        oracle.pattern_sparsified_powers(A, k=2)


def test_diagonal_matrix_gives_diagonal_pattern():
    """A diagonal A has S = 0: every power vector is empty after the first
    product and the pattern is the identity's, for any parameters."""
    n = 25
    A = synth._coo_to_csc(n, np.arange(n), np.arange(n), np.linspace(1.0, 3.0, n))
    for prm in (dict(k=1, tau_i=0.0), dict(k=4, tau_i=0.3, p_l=2)):
        P = oracle.pattern_sparsified_powers(A, **prm)
        assert np.array_equal(P.colptr, np.arange(n + 1)) and np.array_equal(P.rowidx, np.arange(n))


# ---- block diagonal V_0, the final removal and complex A --------------------

def _blocks(n, sizes):
    s = [0]
    q = 0
    while s[-1] < n:
        s.append(min(n, s[-1] + sizes[q % len(sizes)]))
        q += 1
    return np.array(s, dtype=np.int32)


def _block_mask(n, starts):
    M = np.zeros((n, n), dtype=bool)
    for a, b in zip(starts, starts[1:]):
        M[a:b, a:b] = True
    return M


@pytest.mark.parametrize("cplx", [False, True])
def test_unit_blocks_reduce_to_the_diagonal_v0(cplx):
    """Blocks of one row are the diagonal matrices: the block route (LU
    solves) must give the diagonal route's pattern."""
    A = synth.random_small(70, 4, 21, complex_=cplx)
    prm = dict(k=3, tau_i=0.2, p_i=3, tau_l=0.1, p_l=6)
    P0 = oracle.pattern_sparsified_powers(A, **prm)
    P1 = oracle.pattern_sparsified_powers(A, **prm, v0_blocks=np.arange(A.n + 1))
    assert np.array_equal(P0.colptr, P1.colptr) and np.array_equal(P0.rowidx, P1.rowidx)


@pytest.mark.parametrize("cplx", [False, True])
def test_block_S_is_the_dense_inverse_product(cplx):
    """S = V_0^{-1}(A - P_{V_0} A) against a dense inverse (NumPy inv, not
    the oracle's LU solves): column c's rows are every row of the blocks
    its entries outside c's block reach, and nothing in c's own block."""
    A = synth.random_small(48, 5, 8, complex_=cplx)
    starts = _blocks(A.n, [5, 7, 3, 8])
    Ad = dense(A)
    M = _block_mask(A.n, starts)
    V0 = np.where(M, Ad, 0)
    Sd = np.linalg.inv(V0) @ (Ad - V0)
    S = oracle.sparsified_S(A, starts)
    off = (Ad != 0) & ~M
    for c in range(A.n):
        rows, vals = S[c]
        reach = np.zeros(A.n, dtype=bool)
        for i in np.nonzero(off[:, c])[0]:
            reach |= M[i]
        assert list(rows) == list(np.nonzero(reach)[0]), c
        np.testing.assert_allclose(np.array(vals), Sd[rows, c], rtol=0,
                                   atol=1e-11 * max(1.0, np.abs(Sd[:, c]).max()))
        assert np.all(np.abs(Sd[~reach, c]) <= 1e-11 * max(1.0, np.abs(Sd[:, c]).max()))


def test_block_series_without_dropping_is_structural():
    """No dropping: the pattern is that of (I + S)^k, S's structure being the
    blocks reached by the entries outside each column's block, less the rows
    of the column's own block other than j (boolean matrix powers)."""
    A = synth.random_small(60, 3, 4)
    starts = _blocks(A.n, [4, 6])
    M = _block_mask(A.n, starts)
    off = (dense(A) != 0) & ~M
    Sst = (M.astype(np.int64) @ off.astype(np.int64)) > 0
    for k in (1, 2, 3):
        R = np.eye(A.n, dtype=bool)
        acc = R.copy()
        for _ in range(k):
            R = (Sst.astype(np.int64) @ R.astype(np.int64)) > 0
            acc |= R
        acc &= ~M | np.eye(A.n, dtype=bool)
        P = oracle.pattern_sparsified_powers(A, k=k, tau_i=0.0, v0_blocks=starts)
        assert _cols(P) == [list(np.nonzero(acc[:, j])[0]) for j in range(A.n)], k


def test_removal_leaves_only_the_diagonal_inside_each_block():
    """The final step removes V_0's pattern minus the identity: inside its
    block, column j keeps row j only; outside, the rows are those of the
    same run without the removal."""
    A = synth.convdiff(8, 2, 3)
    starts = np.arange(0, A.n + 1, 8, dtype=np.int32)
    lo, hi = starts[:-1].repeat(8), starts[1:].repeat(8)
    prm = dict(k=3, tau_i=0.05, tau_l=0.02)
    got = oracle.sparsified_powers_columns(A, range(A.n), **prm, v0_blocks=starts)
    S = oracle._sp_matrix(A, prm["tau_i"], 0, starts)
    for j in range(A.n):
        rows = list(got[j])
        inside = [r for r in rows if lo[j] <= r < hi[j]]
        assert inside == [j]
        raw = oracle._sp_column(S, j, prm["k"], prm["tau_l"], 0)
        assert [r for r in rows if r != j] == [r for r in raw if not lo[j] <= r < hi[j]]


def test_complex_imaginary_couplings_match_the_real_case():
    """A = I + iB against A = I + B (B without diagonal): S = iB, so every
    magnitude of every power is the real case's exactly (products of
    imaginary units are exact) and the patterns agree, dropping included."""
    R = synth.random_small(80, 4, 13)
    val = R.val.copy()
    diag = R.rowidx == np.repeat(np.arange(R.n), np.diff(R.colptr))
    val[diag] = 1.0
    Ar = synth._coo_to_csc(R.n, R.rowidx, np.repeat(np.arange(R.n), np.diff(R.colptr)), val)
    cval = np.where(diag, 1.0 + 0j, 1j * val)
    Ac = synth._coo_to_csc(R.n, R.rowidx, np.repeat(np.arange(R.n), np.diff(R.colptr)), cval)
    prm = dict(k=3, tau_i=0.15, p_i=3, tau_l=0.05, p_l=5)
    Pr = oracle.pattern_sparsified_powers(Ar, **prm)
    Pc = oracle.pattern_sparsified_powers(Ac, **prm)
    assert _cols(Pr) == _cols(Pc)


def test_margin_is_zero_on_an_exact_tie_and_positive_otherwise():
    """Two off-diagonal entries of equal magnitude compete for one place
    (count rule): the decision is a tie (margin 0, the lower row wins);
    unequal magnitudes give the relative gap."""
    n = 4
    rows = [0, 1, 2, 3, 1, 2, 0, 3]
    cols = [0, 1, 2, 3, 0, 0, 3, 2]
    for v, want in ((0.5, 0.0), (0.25, 0.75)):
        vals = [1.0, 1.0, 1.0, 1.0, 0.5, v, 0.1, 0.1]
        A = synth._coo_to_csc(n, np.array(rows), np.array(cols), np.array(vals))
        out = oracle.sparsified_powers_columns(A, [0], k=1, tau_i=0.0, p_i=1, with_margin=True)
        r, m = out[0]
        assert list(r) == [0, 1]
        assert m == pytest.approx(want)
