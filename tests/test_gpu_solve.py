"""GPU apply M = W V^{-1} and right-preconditioned BiCGSTAB against the oracle.

The GPU path factors, applies and solves with its own factors; the oracle
does the same with its own (CPU) factors on the same matrix.  Iteration
counts must agree within max(1, 5 %), and the GPU's true residual must meet
the tolerance.
"""
import numpy as np
import pytest

import oracle
import synth
from tests._gpu import oracle_pattern, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_1208_3573_amd import diaf
    assert torch.cuda.is_available()
    return diaf.Context(0)


CASES = {
    "convdiff2d_32_gs_v": (lambda: synth.convdiff(32, 2, 1), "A", "gs_upper", 0, "unit_v"),
    "convdiff2d_32_gs_w": (lambda: synth.convdiff(32, 2, 1), "A", "gs_upper", 0, "unit_w"),
    "convdiff3d_16_v": (lambda: synth.convdiff(16, 3, 7), "A2", "topk_lower", 5, "unit_v"),
    "convdiff3d_16_w": (lambda: synth.convdiff(16, 3, 7), "A2", "topk_lower", 5, "unit_w"),
    # complex: with the top-7 triangle rule V comes out numerically singular on
    # this problem (cond ~ 1e17, Section 3.1's warning); the Gauss-Seidel V
    # pattern converges in both modes
    "helmholtz_32_gs_v": (lambda: synth.helmholtz(32, 5.0, 0.5), "A2", "gs_upper", 0, "unit_v"),
    "helmholtz_32_gs_w": (lambda: synth.helmholtz(32, 5.0, 0.5), "A2", "gs_upper", 0, "unit_w"),
    "convdiff3d_64_v": (lambda: synth.workload_matrix("convdiff3d_64"), "A2", "topk_lower", 5,
                        "unit_v"),
    "convdiff3d_64_w": (lambda: synth.workload_matrix("convdiff3d_64"), "A2", "topk_lower", 5,
                        "unit_w"),
    "diag_spai": (lambda: synth.convdiff(16, 3, 8), "A2", "diag", 0, "unit_v"),
}


@pytest.mark.parametrize("name", list(CASES))
def test_bicgstab_iterations_match_oracle(ctx, name):
    import torch
    from paper_1208_3573_amd import diaf
    build, w, v, l, mode = CASES[name]
    A = build()
    b = synth.rhs_ones(A)
    J = oracle_pattern(A, w)
    O = oracle.factor(A, J, mode, v, l)
    upper = v in ("gs_upper", "topk_upper")
    _, oinfo = oracle.bicgstab(A, b, O, upper=upper, tol=1e-8, maxit=1000)
    say(f"case {name}: oracle its={oinfo.iters} flag={oinfo.flag}")
    dA = diaf.DeviceCSC.from_host(A)
    F = diaf.diaf_factor(ctx, dA, diaf.make_spec(w=w, v=v, v_count=l), mode)
    db = torch.from_numpy(b).cuda()
    x = torch.zeros_like(db)
    info = diaf.diaf_solve(ctx, dA, F, db, x, 1e-8, 1000)
    say(f"case {name}: gpu its={info.iters} flag={info.flag} relres={info.relres:.3e} "
        f"true={info.relres_true:.3e} levels={F.levels()}")
    assert info.flag == oinfo.flag == 0
    assert abs(info.iters - oinfo.iters) <= max(1, int(0.05 * oinfo.iters))
    assert info.relres <= 1e-8
    assert info.relres_true <= 1e-7
    xs = x.cpu().numpy()
    assert np.max(np.abs(xs - 1.0)) < 1e-3
    F.close()


def _trailing_growth(V, b, lines, N):
    """max |t| of t = V22^{-1} b2 for the trailing `lines` grid lines of an
    upper triangular V: (V^{-1})'s trailing block is V22^{-1}, so this bounds
    ||V^{-1}|| from below (and kappa(V), with ||V|| >= ||V22||)."""
    import scipy.sparse.linalg as spla
    s0 = V.shape[0] - lines * N
    with np.errstate(all="ignore"):
        t = spla.spsolve_triangular(V[s0:, s0:].tocsr(), b[s0:], lower=False)
    return float(np.max(np.abs(t)))


def test_helmholtz_512_unit_w_topk_upper_outcome(ctx):
    """The Helmholtz workload with unit-norm w and the top-7 upper V: with
    the null-space choice no diagonal entry of V vanishes, but V^{-1} grows
    by about an order of magnitude per grid line (the boundary columns at
    x = 0 have off-diagonal mass up to 28 times the diagonal), so the back
    substitution overflows and BiCGSTAB breaks down in its first iteration,
    on the GPU and in the oracle alike.  The GPU's V gives the lower bound on
    kappa(V) that the test reports."""
    import torch
    from paper_1208_3573_amd import diaf
    cfg = synth.WORKLOADS["helmholtz2d_512"]
    A = synth.workload_matrix("helmholtz2d_512")
    b = synth.rhs_ones(A)
    J = oracle_pattern(A, "A2")
    O = oracle.factor(A, J, "unit_w", "topk_upper", 7)
    _, oinfo = oracle.bicgstab(A, b, O, upper=True, tol=1e-8, maxit=1000)
    dA = diaf.DeviceCSC.from_host(A)
    F = diaf.diaf_factor(ctx, dA, diaf.make_spec(w="A2", v=cfg["v"], v_count=cfg["v_count"]),
                         "unit_w")
    H = F.to_host()
    dvals = np.abs(H["Vval"][H["Vri"] == np.repeat(np.arange(A.n), np.diff(H["Vcp"]))])
    say(f"helmholtz 512: min |v_jj| gpu {dvals.min():.3e}, oracle its={oinfo.iters} "
        f"flag={oinfo.flag}")
    assert dvals.min() > 0.1
    db = torch.from_numpy(b).cuda()
    x = torch.zeros_like(db)
    info = diaf.diaf_solve(ctx, dA, F, db, x, 1e-8, 1000)
    import scipy.sparse as sp
    V = sp.csc_matrix((H["Vval"], H["Vri"], H["Vcp"]), shape=(A.n, A.n))
    growth = {nl: _trailing_growth(V, b, nl, 512) for nl in (4, 8, 16, 32, 64)}
    say(f"helmholtz 512: gpu its={info.iters} flag={info.flag}; max |V22^-1 b| over the "
        f"trailing grid lines {growth}")
    assert oinfo.flag == 2 and info.flag == oinfo.flag and info.iters == oinfo.iters
    # the oracle's V: 6.6, 1.3e3, 6.6e6, 1.4e14, 6.8e28 for 4 ... 64 lines
    assert growth[16] > 1e5 * growth[4] and growth[64] > 1e25


def test_unpreconditioned_bicgstab_matches_oracle(ctx):
    import torch
    from paper_1208_3573_amd import diaf
    A = synth.convdiff(16, 3, 7)
    b = synth.rhs_ones(A)
    _, oinfo = oracle.bicgstab(A, b, None)
    dA = diaf.DeviceCSC.from_host(A)
    db = torch.from_numpy(b).cuda()
    x = torch.zeros_like(db)
    info = diaf.diaf_solve(ctx, dA, None, db, x, 1e-8, 1000)
    assert abs(info.iters - oinfo.iters) <= max(1, int(0.05 * oinfo.iters))
    assert info.flag == 0 and info.relres_true < 1e-7


def test_bicgstab_flags_breakdown_and_maxit(ctx):
    import torch
    import scipy.sparse as sp
    from paper_1208_3573_amd import diaf
    # skew-symmetric plus a tiny diagonal so the diagonal is present: with
    # M = I, <r, A r> = 1e-300 * ||r||^2 underflows the breakdown test
    n = 64
    Ad = np.zeros((n, n))
    for i in range(n - 1):
        Ad[i, i + 1] = 1.0
        Ad[i + 1, i] = -1.0
    np.fill_diagonal(Ad, 1e-320)
    A = synth.CSC.from_scipy(sp.csc_matrix(Ad))
    A.val[A.rowidx == np.repeat(np.arange(n), np.diff(A.colptr))] = 0.0
    dA = diaf.DeviceCSC.from_host(A)
    db = torch.ones(n, dtype=torch.float64, device="cuda")
    x = torch.zeros_like(db)
    info = diaf.diaf_solve(ctx, dA, None, db, x, 1e-8, 100)
    _, oinfo = oracle.bicgstab(A, np.ones(n), None, maxit=100)
    assert info.flag == 2 and oinfo.flag == 2 and info.iters == oinfo.iters == 1
    A = synth.convdiff(16, 2, 2)
    dA = diaf.DeviceCSC.from_host(A)
    db = torch.from_numpy(synth.rhs_ones(A)).cuda()
    x = torch.zeros_like(db)
    info = diaf.diaf_solve(ctx, dA, None, db, x, 1e-8, 3)
    assert info.flag == 1 and info.iters == 3


@pytest.mark.parametrize("cplx", [False, True])
def test_apply_matches_oracle(ctx, cplx):
    import torch
    from paper_1208_3573_amd import diaf
    A = synth.convdiff(12, 3, 3) if not cplx else synth.helmholtz(40, 10.0, 0.5)
    v = "topk_lower" if not cplx else "topk_upper"
    J = oracle_pattern(A, "A2")
    O = oracle.factor(A, J, "unit_v", v, 5)
    rng = np.random.default_rng(0)
    x = rng.standard_normal(A.n) + (1j * rng.standard_normal(A.n) if cplx else 0)
    yo = oracle.apply(O, x, upper=(v == "topk_upper"))
    dA = diaf.DeviceCSC.from_host(A)
    F = diaf.diaf_factor(ctx, dA, diaf.make_spec(w="A2", v=v, v_count=5), "unit_v")
    xd = torch.from_numpy(x).cuda()
    yd = torch.zeros_like(xd)
    diaf.diaf_apply(ctx, F, xd, yd)
    yg = yd.cpu().numpy()
    err = np.linalg.norm(yg - yo) / np.linalg.norm(yo)
    say(f"apply rel err {err:.3e}")
    assert err < 1e-9
    F.close()


def test_singular_v_is_reported(ctx):
    """A V pattern without the diagonal of one column makes V singular: the
    oracle's substitution stops on the zero pivot and the GPU path reports
    DIAF_ESINGULAR (solve flag 3) before any division."""
    import torch
    from paper_1208_3573_amd import diaf
    A = synth.convdiff(8, 2, 1)
    rows, cp = [], [0]
    for j in range(A.n):
        col = [i for i in A.rowidx[A.colptr[j]:A.colptr[j + 1]] if i <= j and not (j == 5 and i == j)]
        rows += col
        cp.append(len(rows))
    Vp = oracle.Pattern(A.n, np.array(cp, np.int32), np.array(rows, np.int32))
    J = oracle.pattern_A(A)
    O = oracle.factor(A, J, "unit_v", "explicit", Vexp=Vp)
    b = synth.rhs_ones(A)
    _, oinfo = oracle.bicgstab(A, b, O, upper=True)
    assert oinfo.flag == 3
    dA = diaf.DeviceCSC.from_host(A)
    dV = diaf.DevicePattern.from_host(Vp.colptr, Vp.rowidx)
    F = diaf.diaf_factor(ctx, dA, diaf.make_spec(w="A", v="explicit", v_explicit=dV), "unit_v")
    db = torch.from_numpy(b).cuda()
    x = torch.zeros_like(db)
    info = diaf.diaf_solve(ctx, dA, F, db, x, 1e-8, 100)
    assert info.flag == 3 and info.iters == oinfo.iters == 1
    assert F.stats().count_zero_pivot == 1
    with pytest.raises(diaf.DiafError) as ei:
        diaf.diaf_apply(ctx, F, db, x)
    assert ei.value.code == diaf.DIAF_ESINGULAR
    F.close()


def test_graph_replay_matches_eager(ctx):
    """The BiCGSTAB batches replayed from one captured graph give the same
    iterate, bit for bit, as the same kernels enqueued one by one; two solves
    in a row with eager work in between keep agreeing."""
    import torch
    from paper_1208_3573_amd import diaf
    A = synth.convdiff(20, 3, 9)
    b = synth.rhs_ones(A)
    dA = diaf.DeviceCSC.from_host(A)
    F = diaf.diaf_factor(ctx, dA, diaf.make_spec(w="A2", v="topk_lower", v_count=5), "unit_v")
    db = torch.from_numpy(b).cuda()
    out = {}
    for graph in (0, 1, 0, 1):
        ctx.set_option("graph", graph)
        x = torch.zeros_like(db)
        info = diaf.diaf_solve(ctx, dA, F, db, x, 1e-8, 500)
        y = torch.empty_like(db)
        diaf.diaf_apply(ctx, F, x, y)  # eager work between the solves
        torch.cuda.synchronize()
        key = (graph, len([k for k in out if k[0] == graph]))
        out[key] = (info.iters, info.flag, x.cpu().numpy())
    ctx.set_option("graph", 1)
    ref = out[(0, 0)]
    for k, v in out.items():
        assert v[0] == ref[0] and v[1] == ref[1] == 0, k
        assert np.array_equal(v[2], ref[2]), k
    F.close()


@pytest.mark.parametrize("cplx", [False, True])
def test_trsv_launch_shapes_agree(ctx, cplx):
    """Every launch shape of the triangular solve (waves per workgroup, i.e.
    rows per chunk) consumes the entries of each row in the same order, so
    W V^{-1} x comes out bit-identical, for lower (real) and upper (complex)
    V, on a chunk count that leaves a ragged last chunk."""
    import torch
    from paper_1208_3573_amd import diaf
    A = synth.convdiff(21, 3, 5) if not cplx else synth.helmholtz(70, 10.0, 0.5)
    v = "topk_lower" if not cplx else "gs_upper"
    dA = diaf.DeviceCSC.from_host(A)
    F = diaf.diaf_factor(ctx, dA, diaf.make_spec(w="A2", v=v, v_count=5), "unit_v")
    rng = np.random.default_rng(1)
    xh = rng.standard_normal(A.n) + (1j * rng.standard_normal(A.n) if cplx else 0)
    xd = torch.from_numpy(xh).cuda()
    ref = None
    for waves in (1, 2, 4, 8, 16):
        ctx.set_option("trsv_waves", waves)
        yd = torch.zeros_like(xd)
        diaf.diaf_apply(ctx, F, xd, yd)
        y = yd.cpu().numpy()
        if ref is None:
            ref = y
        assert np.array_equal(y, ref), waves
    ctx.set_option("trsv_waves", 8)
    F.close()


def _depth(H, lower):
    """Longest chain of rows of a triangular V (pattern of the GPU's own V,
    plain dynamic programming in dependency order)."""
    n = H["n"]
    import scipy.sparse as sp
    R = sp.csc_matrix((np.ones(len(H["Vri"])), H["Vri"], H["Vcp"]), shape=(n, n)).tocsr()
    lev = np.zeros(n, dtype=np.int64)
    order = range(n) if lower else range(n - 1, -1, -1)
    for i in order:
        cols = R.indices[R.indptr[i]:R.indptr[i + 1]]
        deps = cols[cols < i] if lower else cols[cols > i]
        lev[i] = 1 + (lev[deps].max() if deps.size else 0)
    return int(lev.max()) if n else 0


@pytest.mark.parametrize("v,l,lower", [("topk_lower", 5, True), ("gs_upper", 0, False),
                                       ("topk_upper", 4, False), ("diag", 0, None)])
def test_levels_are_the_longest_dependency_chain(ctx, v, l, lower):
    from paper_1208_3573_amd import diaf
    A = synth.convdiff(12, 3, 7)
    dA = diaf.DeviceCSC.from_host(A)
    F = diaf.diaf_factor(ctx, dA, diaf.make_spec(w="A2", v=v, v_count=l), "unit_v")
    assert F.stats().v_levels == 0  # taken on request only
    got = F.levels()
    want = 1 if lower is None else _depth(F.to_host(), lower)
    say(f"V {v}: depth {got}, host walk {want}")
    assert got == want
    assert F.stats().v_levels == got and F.levels() == got
    F.close()
