"""Seeded synthetic workloads for the direct approximate factoring AW ~ V.

This module holds input generators only: it builds sparse matrices in
compressed-sparse-column (CSC) form from a seed, plus the right-hand side
b = A * ones used by the paper's experiments (Section 5: the solution of
the test systems is the all-ones vector).  It contains none of the
factoring, pattern, apply or solver arithmetic; both the CPU oracle and the
GPU library consume its output.

Matrices
--------
* ``convdiff(N, d, seed)``: convection-diffusion on an N^d grid, centred
  finite differences, Dirichlet boundary, h = 1/(N+1), scaled by h^2:
  a_ii = 2d and a_{i, i +- e_k} = -1 +- (h/2) beta_k(x_i), with the
  convection coefficients beta drawn iid uniform in [-20, 20] per node and
  per direction (row i uses its own node's beta).  Natural ordering,
  i = x + N*y + N^2*z.
* ``helmholtz(N, kappa, damping)``: complex shifted 2D Helmholtz,
  h^2(-Lap_h) - (kappa h)^2 (1 - damping*i) I, 5-point, Dirichlet.
* ``random_lognormal(n, seed)``: random nonsymmetric matrix whose column
  degrees are clip(round(LogNormal(mu, sigma)), 3, 200) including the
  diagonal, off-diagonal rows distinct and uniform, values N(0,1); on a
  uniform random 70 % of rows the diagonal is replaced by 1.2 times the
  row's off-diagonal absolute sum.
* ``random_small(n, ...)``: tiny random sparse matrices with a full
  diagonal, for the oracle's pins.
"""
from __future__ import annotations

import functools
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp


@dataclass
class CSC:
    """A square sparse matrix in CSC form: int32 colptr[n+1], int32
    rowidx[nnz] (sorted and unique within each column), values float64 or
    complex128."""

    n: int
    colptr: np.ndarray
    rowidx: np.ndarray
    val: np.ndarray

    @property
    def nnz(self) -> int:
        return int(self.colptr[-1])

    @property
    def is_complex(self) -> bool:
        return np.iscomplexobj(self.val)

    def to_scipy(self) -> sp.csc_matrix:
        return sp.csc_matrix((self.val, self.rowidx, self.colptr), shape=(self.n, self.n))

    @staticmethod
    def from_scipy(m) -> "CSC":
        m = sp.csc_matrix(m)
        m.sum_duplicates()
        m.sort_indices()
        return CSC(
            n=m.shape[0],
            colptr=np.ascontiguousarray(m.indptr, dtype=np.int32),
            rowidx=np.ascontiguousarray(m.indices, dtype=np.int32),
            val=np.ascontiguousarray(m.data),
        )


def _coo_to_csc(n, rows, cols, vals) -> CSC:
    m = sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsc()
    return CSC.from_scipy(m)


def convdiff(N: int, d: int, seed: int, beta_max: float = 20.0) -> CSC:
    """Convection-diffusion operator on an N^d grid (see module docstring)."""
    n = N ** d
    h = 1.0 / (N + 1)
    rng = np.random.default_rng(seed)
    beta = rng.uniform(-beta_max, beta_max, size=(n, d))
    idx = np.arange(n, dtype=np.int64)
    rows = [idx]
    cols = [idx]
    vals = [np.full(n, 2.0 * d)]
    for k in range(d):
        stride = N ** k
        coord = (idx // stride) % N
        up = coord < N - 1
        dn = coord > 0
        rows += [idx[up], idx[dn]]
        cols += [idx[up] + stride, idx[dn] - stride]
        vals += [-1.0 + 0.5 * h * beta[up, k], -1.0 - 0.5 * h * beta[dn, k]]
    return _coo_to_csc(n, np.concatenate(rows), np.concatenate(cols), np.concatenate(vals))


def helmholtz(N: int = 512, kappa: float = 40.0, damping: float = 0.5) -> CSC:
    """Complex shifted 2D Helmholtz operator, 5-point, Dirichlet, scaled by h^2."""
    n = N * N
    h = 1.0 / (N + 1)
    idx = np.arange(n, dtype=np.int64)
    diag = 4.0 - (kappa * h) ** 2 * (1.0 - 1j * damping)
    rows = [idx]
    cols = [idx]
    vals = [np.full(n, diag, dtype=np.complex128)]
    for k in range(2):
        stride = N ** k
        coord = (idx // stride) % N
        for mask, off in ((coord < N - 1, stride), (coord > 0, -stride)):
            rows.append(idx[mask])
            cols.append(idx[mask] + off)
            vals.append(np.full(int(mask.sum()), -1.0 + 0j))
    return _coo_to_csc(n, np.concatenate(rows), np.concatenate(cols), np.concatenate(vals))


def random_lognormal(n: int, seed: int, mu: float = 2.3, sigma: float = 0.8,
                     lo: int = 3, hi: int = 200, boost_frac: float = 0.7,
                     boost: float = 1.2) -> CSC:
    """Random nonsymmetric sparse matrix with lognormal column degrees."""
    rng = np.random.default_rng(seed)
    deg = np.clip(np.rint(rng.lognormal(mu, sigma, n)), lo, hi).astype(np.int64)
    cols = np.repeat(np.arange(n, dtype=np.int64), deg - 1)
    rows = rng.integers(0, n, size=cols.size, dtype=np.int64)
    # Redraw rows that hit the diagonal or repeat within their column until
    # every column has distinct off-diagonal rows.
    while True:
        key = cols * n + rows
        order = np.argsort(key, kind="stable")
        dup = np.zeros(cols.size, dtype=bool)
        ks = key[order]
        dup[order[1:]] = ks[1:] == ks[:-1]
        bad = dup | (rows == cols)
        nbad = int(bad.sum())
        if nbad == 0:
            break
        rows[bad] = rng.integers(0, n, size=nbad, dtype=np.int64)
    offval = rng.standard_normal(cols.size)
    dval = rng.standard_normal(n)
    rowsum = np.bincount(rows, weights=np.abs(offval), minlength=n)
    boosted = rng.permutation(n)[: int(round(boost_frac * n))]
    sel = boosted[rowsum[boosted] > 0]
    dval[sel] = boost * rowsum[sel]
    idx = np.arange(n, dtype=np.int64)
    return _coo_to_csc(n, np.concatenate([rows, idx]), np.concatenate([cols, idx]),
                       np.concatenate([offval, dval]))


def random_small(n: int, per_col: int, seed: int, complex_: bool = False,
                 diag_shift: float = 0.0) -> CSC:
    """Tiny random sparse matrix with a full diagonal and ``per_col``
    off-diagonal entries per column (distinct rows), values N(0,1)."""
    rng = np.random.default_rng(seed)
    rows, cols = [], []
    for j in range(n):
        others = np.setdiff1d(np.arange(n), [j])
        pick = rng.choice(others, size=min(per_col, n - 1), replace=False)
        rows += [j] + list(pick)
        cols += [j] * (1 + len(pick))
    rows = np.array(rows)
    cols = np.array(cols)
    v = rng.standard_normal(rows.size)
    if complex_:
        v = v + 1j * rng.standard_normal(rows.size)
    v[rows == cols] += diag_shift
    return _coo_to_csc(n, rows, cols, v)


def rhs_ones(A: CSC) -> np.ndarray:
    """b = A * ones: the test right-hand side whose exact solution is the
    all-ones vector."""
    return np.asarray(A.to_scipy() @ np.ones(A.n, dtype=A.val.dtype))


# ---------------------------------------------------------------------------
# Named workloads.  Each entry names the matrix, the W and V pattern rules,
# the norm modes and the solve settings used for it.
# ---------------------------------------------------------------------------

WORKLOADS = {
    "convdiff2d_32": dict(kind="convdiff", N=32, d=2, seed=1, w="A", v="gs_upper", v_count=0,
                          modes=("unit_v", "unit_w")),
    "convdiff3d_64": dict(kind="convdiff", N=64, d=3, seed=2, w="A2", v="topk_lower", v_count=5,
                          modes=("unit_v", "unit_w")),
    "random_1m": dict(kind="random", n=1_000_000, seed=3, w="A_1hop_topk", w_topk=8,
                      v="topk_lower", v_count=5, modes=("unit_v", "unit_w")),
    "helmholtz2d_512": dict(kind="helmholtz", N=512, kappa=40.0, damping=0.5, w="A2",
                            v="topk_upper", v_count=7, modes=("unit_w",)),
    "convdiff3d_48_train": dict(kind="convdiff", N=48, d=3, seed=5000, w="A2", v="topk_lower",
                                v_count=5, modes=("unit_w", "unit_v")),
}


@functools.lru_cache(maxsize=4)
def workload_matrix(name: str, seed: int | None = None) -> CSC:
    """Build (and cache in-process) the matrix of a named workload."""
    w = WORKLOADS[name]
    s = w.get("seed") if seed is None else seed
    if w["kind"] == "convdiff":
        return convdiff(w["N"], w["d"], s)
    if w["kind"] == "helmholtz":
        return helmholtz(w["N"], w["kappa"], w["damping"])
    if w["kind"] == "random":
        return random_lognormal(w["n"], s)
    raise KeyError(name)
