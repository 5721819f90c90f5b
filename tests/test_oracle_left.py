"""Pins of the oracle's left variant (the remarks of Section 4: a left
approximate factoring W A ~ V of the inverse, M = V^{-1} W, used from the
left): the columnwise method on A^*, its transposition, the apply order and
the left-preconditioned BiCGSTAB.

The checks use SciPy products and triangular solves, SciPy's BiCGSTAB on
the explicitly left-preconditioned operator, and the exact case, not the
oracle's own routines.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle
import synth


def _left(A, w, v, l, mode):
    Ah = oracle.conj_transpose(A)
    J = oracle.pattern_A2(Ah) if w == "A2" else oracle.pattern_A(Ah)
    Ft = oracle.factor(Ah, J, mode, v, l)
    return Ah, Ft, oracle.left_factors(Ft)


@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("mode", ["unit_v", "unit_w"])
def test_row_residuals_of_w_a_minus_v(cplx, mode):
    """r_j of the factors of A^* are the row norms of W A - V with
    W = W~^*, V = V~^*; a transpose without the conjugate fails this for
    complex A."""
    A = synth.random_small(80, 4, 5, complex_=cplx, diag_shift=1.0)
    _, Ft, F = _left(A, "A2", "topk_lower", 4, mode)
    R = (F.W_scipy() @ A.to_scipy() - F.V_scipy()).toarray()
    rown = np.linalg.norm(R, axis=1)
    ok = np.isfinite(Ft.r)
    assert np.allclose(rown[ok], Ft.r[ok], rtol=1e-9, atol=1e-12)
    # V is upper triangular: the lower rule on A^* transposes to the upper side
    assert sp.tril(F.V_scipy(), -1).nnz == 0


@pytest.mark.parametrize("cplx", [False, True])
def test_left_apply_order(cplx):
    """apply(left) is V^{-1} (W x) (SciPy product then SciPy triangular
    solve), not W V^{-1} x."""
    A = synth.random_small(60, 4, 6, complex_=cplx, diag_shift=2.0)
    _, _, F = _left(A, "A", "topk_lower", 3, "unit_v")
    rng = np.random.default_rng(0)
    x = rng.standard_normal(A.n) + (1j * rng.standard_normal(A.n) if cplx else 0)
    y = oracle.apply(F, x, True, left=True)
    ref = spla.spsolve_triangular(F.V_scipy().tocsr(), F.W_scipy() @ x, lower=False)
    assert np.linalg.norm(y - ref) <= 1e-12 * np.linalg.norm(ref)
    other = F.W_scipy() @ spla.spsolve_triangular(F.V_scipy().tocsr(), x, lower=False)
    assert np.linalg.norm(y - other) > 1e-6 * np.linalg.norm(ref)


def test_exact_case_left_inverse():
    """A full W pattern with the diagonal V gives V^{-1} W = A^{-1} from the
    left as well (Appendix A.4 applied to A^*)."""
    A = synth.random_small(12, 3, 2, diag_shift=2.0)
    n = A.n
    Ah = oracle.conj_transpose(A)
    full = oracle.Pattern(n, np.arange(0, n * n + 1, n, dtype=np.int32),
                          np.tile(np.arange(n, dtype=np.int32), n))
    F = oracle.left_factors(oracle.factor(Ah, full, "unit_v", "diag"))
    M = np.linalg.solve(F.V_scipy().toarray(), F.W_scipy().toarray())
    assert np.allclose(M @ A.to_scipy().toarray(), np.eye(n), atol=1e-10)


@pytest.mark.parametrize("mode", ["unit_v", "unit_w"])
def test_left_bicgstab_matches_scipy(mode):
    """Left preconditioning is BiCGSTAB without a preconditioner on the
    operator M A and the right-hand side M b: SciPy's BiCGSTAB on that
    operator (with M from SciPy solves) stops within one iteration of the
    oracle (the half-step convention).  The stop test is on the
    preconditioned residual, which the returned x meets; the true residual
    is reported as computed, and can be much larger (unit-norm v here:
    7e-5 against 1e-8), the difference the paper's remark on left and right
    approximate inverses points at."""
    A = synth.convdiff(24, 2, 1)
    b = synth.rhs_ones(A)
    _, _, F = _left(A, "A2", "topk_lower", 4, mode)
    x, info = oracle.bicgstab(A, b, F, upper=True, tol=1e-8, maxit=1000, left=True)
    W = F.W_scipy().tocsr()
    Vr = F.V_scipy().tocsr()
    As = A.to_scipy().tocsr()
    M = lambda z: spla.spsolve_triangular(Vr, W @ z, lower=False)
    op = spla.LinearOperator(As.shape, matvec=lambda z: M(As @ z))
    its = [0]
    xs, flag = spla.bicgstab(op, M(b), rtol=1e-8, atol=0.0, maxiter=1000,
                             callback=lambda xk: its.__setitem__(0, its[0] + 1))
    assert flag == 0 and info.flag == 0
    assert abs(its[0] - info.iters) <= 1
    Mb = M(b)
    assert np.linalg.norm(M(b - As @ x)) <= 1.01e-8 * np.linalg.norm(Mb)
    rt = np.linalg.norm(b - As @ x) / np.linalg.norm(b)
    assert abs(info.relres_true - rt) <= 1e-6 * rt
    assert np.allclose(x, 1.0, atol=1e-3)
