"""GPU kernels of the learned W-pattern proposer against the FP64 reference.

Features and labels are checked element by element, the MLP forward and the
loss gradient against the FP64 back-propagation (FP32 tolerances), training
must lower the loss, and the residual gate must behave at its limits:
a negative gate sends every column back to pattern(A^2) and reproduces the plain
factorization bit for bit, gate infinity keeps the proposal.
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import learned as L
from tests._gpu import compare, oracle_pattern, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_1208_3573_amd import diaf
    assert torch.cuda.is_available()
    return diaf.Context(0)


def _cand(A):
    J = oracle_pattern(A, "A2")
    return J


@pytest.mark.parametrize("cplx", [False, True])
def test_features_match_reference(ctx, cplx):
    import torch
    from paper_1208_3573_amd import diaf
    A = synth.convdiff(6, 3, 4) if not cplx else synth.helmholtz(12, 5.0, 0.5)
    C = _cand(A)
    ref = L.features(A, C.colptr, C.rowidx).astype(np.float32)
    dA = diaf.DeviceCSC.from_host(A)
    dC = diaf.DevicePattern.from_host(C.colptr, C.rowidx)
    feat = torch.zeros(C.nnz * 16, dtype=torch.float32, device="cuda")
    diaf.diaf_features(ctx, dA, dC, feat)
    got = feat.cpu().numpy().reshape(-1, 16)
    err = np.max(np.abs(got - ref) / np.maximum(1.0, np.abs(ref)))
    say(f"features max err {err:.3e}")
    assert err <= 2e-7


def test_labels_match_reference(ctx):
    import torch
    from paper_1208_3573_amd import diaf
    A = synth.convdiff(8, 3, 5)
    dA = diaf.DeviceCSC.from_host(A)
    F = diaf.diaf_factor(ctx, dA, diaf.make_spec(w="A2", v="topk_lower", v_count=5), "unit_w")
    H = F.to_host()
    lab = torch.zeros(len(H["Wri"]), dtype=torch.float32, device="cuda")
    diaf.diaf_labels(ctx, dA, F, 0.1, lab)
    ref = L.labels(A, H["Wcp"], H["Wri"], H["Wval"], 0.1)
    assert np.array_equal(lab.cpu().numpy(), ref.astype(np.float32))
    F.close()


def test_mlp_forward_and_gradient_match_fp64(ctx):
    import torch
    from paper_1208_3573_amd import diaf
    rng = np.random.default_rng(1)
    theta = L.init_params(7)
    N = 1000
    X = rng.standard_normal((N, 16)).astype(np.float32)
    y = (rng.random(N) < 0.3).astype(np.float32)
    m = diaf.Model(ctx, theta)
    assert np.array_equal(m.params(), theta)
    Xd = torch.from_numpy(X).cuda()
    yd = torch.from_numpy(y).cuda()
    sc = torch.zeros(N, dtype=torch.float32, device="cuda")
    diaf.diaf_mlp_forward(ctx, m, Xd, N, sc)
    sref = L.forward(theta.astype(np.float64), X.astype(np.float64))
    assert np.max(np.abs(sc.cpu().numpy() - sref)) <= 1e-4 * max(1.0, np.abs(sref).max())
    g = torch.zeros(L.NPARAM, dtype=torch.float32, device="cuda")
    loss = diaf.diaf_mlp_loss_grad(ctx, m, Xd, yd, N, g)
    lref, gref = L.loss_grad(theta.astype(np.float64), X.astype(np.float64), y.astype(np.float64))
    gg = g.cpu().numpy()
    rel = np.linalg.norm(gg - gref) / np.linalg.norm(gref)
    say(f"loss {loss:.6f} ref {lref:.6f} grad rel err {rel:.3e}")
    assert abs(loss - lref) <= 1e-5 * max(1.0, lref)
    assert rel <= 1e-4
    m.close()


def test_training_lowers_the_loss(ctx):
    import torch
    from paper_1208_3573_amd import diaf
    A = synth.convdiff(10, 3, 21)
    dA = diaf.DeviceCSC.from_host(A)
    F = diaf.diaf_factor(ctx, dA, diaf.make_spec(w="A2", v="topk_lower", v_count=5), "unit_w")
    H = F.to_host()
    C = diaf.DevicePattern.from_host(H["Wcp"], H["Wri"])
    npairs = len(H["Wri"])
    feat = torch.zeros(npairs * 16, dtype=torch.float32, device="cuda")
    diaf.diaf_features(ctx, dA, C, feat)
    lab = torch.zeros(npairs, dtype=torch.float32, device="cuda")
    diaf.diaf_labels(ctx, dA, F, 0.1, lab)
    m = diaf.Model(ctx, L.init_params(0))
    losses = [diaf.diaf_mlp_train_step(ctx, m, feat, lab, npairs, 3e-3) for _ in range(150)]
    say(f"loss {losses[0]:.4f} -> {losses[-1]:.4f}")
    assert losses[-1] < 0.6 * losses[0]
    m.close()
    F.close()


def test_gate_limits(ctx):
    """gate -1: every column falls back to pattern(A^2) and the result equals
    the plain factorization bit for bit; gate inf: nothing falls back."""
    from paper_1208_3573_amd import diaf
    A = synth.convdiff(10, 3, 3)
    dA = diaf.DeviceCSC.from_host(A)
    m = diaf.Model(ctx, L.init_params(5))
    plain = diaf.diaf_factor(ctx, dA, diaf.make_spec(w="A2", v="topk_lower", v_count=5), "unit_w")
    P = plain.to_host()
    Fz = diaf.diaf_factor(ctx, dA, diaf.make_spec(w="learned", v="topk_lower", v_count=5, model=m,
                                                  gate_tau=-1.0), "unit_w")
    Z = Fz.to_host()
    assert np.all(Z["flags"] & diaf.FLAG_FELL_BACK)
    for key in ("Wcp", "Wri", "Wval", "Vcp", "Vri", "Vval", "r"):
        assert np.array_equal(P[key], Z[key]), key
    Fi = diaf.diaf_factor(ctx, dA, diaf.make_spec(w="learned", v="topk_lower", v_count=5, model=m,
                                                  gate_tau=float("inf")), "unit_w")
    I = Fi.to_host()
    assert not np.any(I["flags"] & diaf.FLAG_FELL_BACK)
    # the learned W pattern is a subset of pattern(A^2) containing the diagonal
    C = oracle_pattern(A, "A2")
    for j in range(A.n):
        rows = set(I["Wri"][I["Wcp"][j]:I["Wcp"][j + 1]])
        assert j in rows
        assert rows <= set(C.rowidx[C.colptr[j]:C.colptr[j + 1]])
    for F in (plain, Fz, Fi):
        F.close()
    m.close()


@pytest.mark.parametrize("mode", ["unit_v", "unit_w"])
def test_trained_proposer_with_partial_fallback(ctx, mode):
    """The committed network on a held-out 3D problem (24^3, seed 77): the
    columns whose proposal fails a gate are refactored with pattern(A^2) and
    merged with the accepted ones.  The merged W and V must reproduce every
    stored residual ||A w_j - v_j|| on the host, every column whose proposal
    was accepted must pass both gates, and the preconditioned BiCGSTAB must
    converge.  With an unreachable dominance gate every column with an
    off-diagonal V entry falls back."""
    import scipy.sparse as sp
    import torch
    from paper_1208_3573_amd import diaf
    from paper_1208_3573_amd import learned as LR
    A = synth.convdiff(24, 3, 77)
    dA = diaf.DeviceCSC.from_host(A)
    model, gate, gate_dom = LR.load(ctx, LR.weights_path(mode))
    spec = diaf.make_spec(w="learned", v="topk_lower", v_count=5, model=model, gate_tau=gate,
                          gate_dom=gate_dom)
    F = diaf.diaf_factor(ctx, dA, spec, mode)
    H = F.to_host()
    n = A.n
    W = sp.csc_matrix((H["Wval"], H["Wri"], H["Wcp"]), shape=(n, n))
    V = sp.csc_matrix((H["Vval"], H["Vri"], H["Vcp"]), shape=(n, n))
    R = (A.to_scipy().tocsc() @ W - V).tocsc()
    rh = np.sqrt(np.asarray(R.multiply(R).sum(axis=0)).ravel())
    assert np.max(np.abs(rh - H["r"])) <= 1e-12 * (1.0 + np.max(H["r"]))
    fb = (H["flags"] & diaf.FLAG_FELL_BACK) != 0
    s = np.ones(n) if mode == "unit_v" else LR._block_fro(A, H["Wcp"], H["Wri"])
    acc = ~fb
    assert np.all(H["r"][acc] / s[acc] <= gate)
    assert np.all(LR._dominance(H)[acc] >= gate_dom)
    say(f"{mode}: fell back {int(fb.sum())} of {n}, nnz(W) {len(H['Wri'])}")
    b = torch.from_numpy(synth.rhs_ones(A)).cuda()
    x = torch.zeros_like(b)
    info = diaf.diaf_solve(ctx, dA, F, b, x, 1e-8, 1000)
    assert info.flag == 0 and info.relres_true <= 1e-7
    F.close()
    spec_all = diaf.make_spec(w="learned", v="topk_lower", v_count=5, model=model, gate_tau=gate,
                              gate_dom=1e300)
    Fa = diaf.diaf_factor(ctx, dA, spec_all, mode)
    Ha = Fa.to_host()
    kept = (Ha["flags"] & diaf.FLAG_FELL_BACK) == 0
    # only columns whose V column has no off-diagonal entry (infinitely
    # dominant) can pass an unreachable dominance gate
    assert np.all(np.isinf(LR._dominance(Ha)[kept]))
    assert kept.sum() < n // 100
    Fa.close()
    model.close()


def test_proposed_pattern_matches_reference_forward(ctx):
    """J_j from the GPU's features and FP32 MLP against J_j from the FP64
    reference features and forward pass with the same rule ({j} plus the
    candidates of pattern(A^2) with score >= 0), using the committed
    network.  Pairs whose FP64 score lies within the FP32 error band of 0
    (1e-4 max(1, max |s|), the forward test's tolerance) may go either way;
    every other pair must agree."""
    from paper_1208_3573_amd import diaf
    from paper_1208_3573_amd import learned as LR
    A = synth.convdiff(12, 3, 5)
    dA = diaf.DeviceCSC.from_host(A)
    model, _, _ = LR.load(ctx, LR.weights_path("unit_v"))
    theta = model.params().astype(np.float64)
    ctx.set_option("gate_small_diag", 0)
    try:
        F = diaf.diaf_factor(ctx, dA, diaf.make_spec(w="learned", v="topk_lower", v_count=5,
                                                     model=model, gate_tau=float("inf")),
                             "unit_v")
    finally:
        ctx.set_option("gate_small_diag", 1)
    H = F.to_host()
    assert not np.any(H["flags"] & diaf.FLAG_FELL_BACK)
    C = oracle_pattern(A, "A2")
    s = L.forward(theta, L.features(A, C.colptr, C.rowidx))
    band = 1e-4 * max(1.0, float(np.abs(s).max()))
    diag = C.rowidx == np.repeat(np.arange(A.n), np.diff(C.colptr))
    keep = (s >= 0) | diag
    ambiguous = (np.abs(s) <= band) & ~diag
    mism = 0
    for j in range(A.n):
        sl = slice(C.colptr[j], C.colptr[j + 1])
        cand = C.rowidx[sl]
        got = np.isin(cand, H["Wri"][H["Wcp"][j]:H["Wcp"][j + 1]])
        bad = (got != keep[sl]) & ~ambiguous[sl]
        mism += int(bad.sum())
    say(f"proposal: {int(keep.sum())} of {C.nnz} pairs kept, {int(ambiguous.sum())} within the "
        f"FP32 band of 0, {mism} disagreements outside it")
    assert mism == 0
    assert ambiguous.sum() <= 1e-3 * C.nnz
    F.close()
    model.close()


@pytest.mark.parametrize("mode", ["unit_v", "unit_w"])
def test_merged_learned_factors_match_oracle(ctx, mode):
    """The learned factorization after the gates (accepted proposals plus the
    columns refactored with pattern(A^2)) against the oracle's factoring on
    the final W pattern: identical V patterns, residuals and singular
    vectors within the parity bars, flags in agreement.  The columns that
    fell back carry exactly pattern(A^2)."""
    from paper_1208_3573_amd import diaf
    from paper_1208_3573_amd import learned as LR
    A = synth.convdiff(24, 3, 77)
    dA = diaf.DeviceCSC.from_host(A)
    model, gate, gate_dom = LR.load(ctx, LR.weights_path(mode))
    spec = diaf.make_spec(w="learned", v="topk_lower", v_count=5, model=model, gate_tau=gate,
                          gate_dom=gate_dom)
    F = diaf.diaf_factor(ctx, dA, spec, mode)
    H = F.to_host()
    fb = np.flatnonzero(H["flags"] & diaf.FLAG_FELL_BACK)
    C = oracle_pattern(A, "A2")
    for j in fb:
        assert np.array_equal(H["Wri"][H["Wcp"][j]:H["Wcp"][j + 1]],
                              C.rowidx[C.colptr[j]:C.colptr[j + 1]])
    Jf = oracle.Pattern(A.n, H["Wcp"].astype(np.int32), H["Wri"].astype(np.int32))
    O = oracle.factor(A, Jf, mode, "topk_lower", 5)
    say(f"{mode}: {fb.size} columns fell back")
    summ = compare(H, Jf, O, A, mode)
    assert summ["excluded"] <= 0.01 * A.n
    F.close()
    model.close()


def test_adam_steps_match_reference(ctx):
    """Two GPU Adam steps against oracle/learned.adam_step fed the same
    gradients (the GPU's own, which the gradient test pins to the FP64
    back-propagation).  FP32 arithmetic and constants (0.999f is not 0.999)
    bound the difference by 1e-6 |theta| + 2e-5 lr."""
    import torch
    from paper_1208_3573_amd import diaf
    rng = np.random.default_rng(3)
    theta = L.init_params(11)
    N = 2000
    X = torch.from_numpy(rng.standard_normal((N, 16)).astype(np.float32)).cuda()
    y = torch.from_numpy((rng.random(N) < 0.3).astype(np.float32)).cuda()
    m = diaf.Model(ctx, theta)
    lr = 3e-3
    th = theta.astype(np.float64)
    mom = np.zeros(L.NPARAM)
    vel = np.zeros(L.NPARAM)
    for step in (1, 2):
        g = torch.zeros(L.NPARAM, dtype=torch.float32, device="cuda")
        diaf.diaf_mlp_loss_grad(ctx, m, X, y, N, g)
        gh = g.cpu().numpy().astype(np.float64)
        diaf.diaf_mlp_train_step(ctx, m, X, y, N, lr)
        th, mom, vel = L.adam_step(th, gh, mom, vel, step, lr)
        got = m.params().astype(np.float64)
        err = np.abs(got - th)
        bound = 1e-6 * np.abs(th) + 2e-5 * lr
        say(f"adam step {step}: max |theta_gpu - theta_ref| {err.max():.3e}")
        assert np.all(err <= bound), (step, float(np.max(err - bound)))
        th = got  # continue from the GPU's parameters (FP32)
    m.close()


def test_learned_gain_with_block_v(ctx):
    """What the trained network gains, on the held-out 64^3 workload (the
    training set is 48^3, seeds from 5000): second basic algorithm, V block
    diagonal on the x-lines, BiCGSTAB to 1e-8 for each W.  The network
    trained on labels at dropping tolerance 0.1 proposes, with no gate, a W
    less than half as dense as pattern(A^2) that still converges; it is
    compared, and its time reported, against plain pattern(A^2) and plain
    pattern(A).  On this workload its proposal is pattern(A) itself, so it
    gains the sparser pattern over pattern(A^2) and loses the inference time
    against pattern(A)."""
    import time
    import torch
    from paper_1208_3573_amd import diaf
    from paper_1208_3573_amd import learned as LR
    A = synth.workload_matrix("convdiff3d_64")
    dA = diaf.DeviceCSC.from_host(A)
    b = torch.from_numpy(synth.rhs_ones(A)).cuda()
    x = torch.zeros_like(b)
    vb = torch.arange(0, A.n + 1, 64, dtype=torch.int32, device="cuda")
    model, _gate, _gdom = LR.load(ctx, LR.weights_path("unit_w", "block"))

    def run(spec):
        best = None
        for _ in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            F = diaf.diaf_factor(ctx, dA, spec, "unit_w")
            info = diaf.diaf_solve(ctx, dA, F, b, x, 1e-8, 1000)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3
            H = F.to_host()
            F.close()
            best = ms if best is None else min(best, ms)
        return best, info, H

    t2, i2, H2 = run(diaf.make_spec(w="A2", v="block", v_blocks=vb))
    t1, i1, H1 = run(diaf.make_spec(w="A", v="block", v_blocks=vb))
    tl, il, HL = run(diaf.make_spec(w="learned", v="block", v_blocks=vb, model=model))
    model.close()
    for info in (i2, i1, il):
        assert info.flag == 0 and info.relres_true <= 1e-7
    assert len(HL["Wri"]) <= 0.5 * len(H2["Wri"])
    same_as_A = (np.array_equal(HL["Wcp"], H1["Wcp"]) and np.array_equal(HL["Wri"], H1["Wri"]))
    say(f"64^3 unit w, block V: pattern(A^2) {t2:.1f} ms / {i2.iters} its / nnz {len(H2['Wri'])}; "
        f"pattern(A) {t1:.1f} ms / {i1.iters} its / nnz {len(H1['Wri'])}; learned {tl:.1f} ms / "
        f"{il.iters} its / nnz {len(HL['Wri'])} (pattern(A): {same_as_A}); gain over "
        f"pattern(A^2) {t2 - tl:+.1f} ms, over pattern(A) {t1 - tl:+.1f} ms")
