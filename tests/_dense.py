"""Independent dense NumPy/SciPy formulations used to pin the oracle.

These use LAPACK (least squares, SVD, inverse) and SciPy routines that the C
oracle does not use, on the dense n x k matrix A(:, J_j) itself rather than
on the oracle's compacted block.
"""
import numpy as np
import scipy.sparse as sp


def dense(A):
    return A.to_scipy().toarray()


def cols_of(P, j):
    return P.rowidx[P.colptr[j]:P.colptr[j + 1]]


def Aj(Ad, J, j):
    """A_j: the columns J_j of dense A (n x k), as the paper defines it."""
    return Ad[:, cols_of(J, j)]


def sin_angle(x, y):
    """sin of the angle between span{x} and span{y}, projection form."""
    x = np.asarray(x).ravel()
    y = np.asarray(y).ravel()
    ny = np.vdot(y, y).real
    if ny == 0:
        return 1.0 if np.linalg.norm(x) > 0 else 0.0
    res = x - y * (np.vdot(y, x) / ny)
    nx = np.linalg.norm(x)
    return float(np.linalg.norm(res) / nx) if nx > 0 else 0.0


def v_of(F, j):
    sl = slice(F.Vcp[j], F.Vcp[j + 1])
    return F.Vri[sl], F.Vval[sl]


def w_of(F, j):
    sl = slice(F.Jcp[j], F.Jcp[j + 1])
    return F.Jri[sl], F.Wval[sl]


def spaiq_lstsq(Ad, J, j):
    """Least-squares column min ||A_j w - e_j|| via LAPACK gelsd."""
    A_j = Aj(Ad, J, j)
    e = np.zeros(Ad.shape[0], dtype=Ad.dtype)
    e[j] = 1
    return np.linalg.lstsq(A_j, e, rcond=None)[0]


def smallest_right_sv(Ad, J, j, L):
    """Right singular vector of sigma_min of A_j with the rows L removed."""
    A_j = Aj(Ad, J, j)
    keep = np.setdiff1d(np.arange(Ad.shape[0]), L)
    U, s, Vh = np.linalg.svd(A_j[keep, :], full_matrices=True)
    return Vh[-1].conj(), s


def trsv_scipy(V, x, upper):
    Vc = sp.csr_matrix(V)
    return sp.linalg.spsolve_triangular(Vc, x, lower=not upper)
