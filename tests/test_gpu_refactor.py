"""diaf_refactor: new values written into the matrix the factors were built
from, same pattern.  The first refactor runs the factor launches eagerly
and records them; for unit-norm v later ones replay them as one captured
graph.  Every refactor must equal a fresh diaf_factor on the same values bit
for bit, with the program's own eager work (fresh factorizations, applies,
synchronizations) between the replays."""
import numpy as np
import pytest

import synth
from tests._gpu import say

pytestmark = pytest.mark.gpu

KEYS = ("Wcp", "Wri", "Wval", "Vcp", "Vri", "Vval", "r", "flags", "lcount")


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_1208_3573_amd import diaf
    assert torch.cuda.is_available()
    return diaf.Context(0)


def _perturbed(A, seed):
    """Same pattern, new values: every entry scaled by a random factor in
    [0.8, 1.2] (the diagonal kept dominant as in the original)."""
    rng = np.random.default_rng(seed)
    f = rng.uniform(0.8, 1.2, size=A.val.shape)
    return A.val * f


CASES = {
    "convdiff3d_16 unit_v A2 topk_lower": (lambda: synth.convdiff(16, 3, 3), "A2", "topk_lower",
                                            5, "unit_v"),
    # pattern(A) of the lognormal matrix: columns for all three factor kernels
    "random_3k unit_v A topk_lower": (lambda: synth.random_lognormal(3000, 7), "A",
                                      "topk_lower", 5, "unit_v"),
    "convdiff3d_12 unit_w A2 topk_lower": (lambda: synth.convdiff(12, 3, 5), "A2", "topk_lower",
                                           5, "unit_w"),
    "helmholtz_16 unit_w A gs_upper": (lambda: synth.helmholtz(16), "A", "gs_upper", 0,
                                       "unit_w"),
}


@pytest.mark.parametrize("name", list(CASES))
def test_refactor_equals_fresh_factor(ctx, name):
    import torch
    from paper_1208_3573_amd import diaf
    mk, w, v, l, mode = CASES[name]
    A = mk()
    dA = diaf.DeviceCSC.from_host(A)
    spec = diaf.make_spec(w=w, v=v, v_count=l)
    F = diaf.diaf_factor(ctx, dA, spec, mode)
    x = torch.ones(A.n, dtype=dA.torch_dtype, device="cuda")
    y = torch.zeros_like(x)
    for rep, seed in enumerate((1, 2, 3, 4)):
        vals = _perturbed(A, seed)
        say(f"case {name}: refactor {rep} (seed {seed})")
        dA.val.copy_(torch.from_numpy(vals).cuda())
        diaf.diaf_refactor(ctx, dA, F)
        H = F.to_host()
        diaf.diaf_apply(ctx, F, x, y)  # apply structures rebuilt from the new values
        torch.cuda.synchronize()
        Fr = diaf.diaf_factor(ctx, dA, spec, mode)
        Hr = Fr.to_host()
        yr = torch.zeros_like(x)
        diaf.diaf_apply(ctx, Fr, x, yr)
        torch.cuda.synchronize()
        for key in KEYS:
            assert np.array_equal(np.asarray(H[key]), np.asarray(Hr[key])), (rep, key)
        assert torch.equal(y, yr), rep
        st = F.stats()
        say(f"  factor pass {st.ms_factor:.3f} ms (fresh {Fr.stats().ms_factor:.3f} ms), "
            f"nnz(V) {st.nnz_v}, ||AW - V|| {st.nrm:.4g}, columns small/mid/generic "
            f"{st.cols_small}/{st.cols_mid}/{sum(st.cols_generic_class)}")
        Fr.close()
    F.close()


def test_refactor_errors(ctx):
    import torch
    from paper_1208_3573_amd import diaf
    A = synth.convdiff(10, 3, 1)
    dA = diaf.DeviceCSC.from_host(A)
    F = diaf.diaf_factor(ctx, dA, diaf.make_spec(w="A2", v="topk_lower", v_count=4), "unit_v")
    say("case other value buffer")
    dB = diaf.DeviceCSC(A.n, dA.colptr, dA.rowidx, dA.val.clone())
    with pytest.raises(diaf.DiafError) as ei:
        diaf.diaf_refactor(ctx, dB, F)
    assert ei.value.code == diaf.DIAF_EINVAL
    say("case pattern changed in place")
    B = synth.convdiff(10, 3, 1)
    rows = B.rowidx.copy()
    # move one off-diagonal entry of column 5 to another row not in the column
    c0, c1 = B.colptr[5], B.colptr[6]
    col = list(rows[c0:c1])
    free = [r for r in range(A.n) if r not in col]
    off = [q for q in range(c0, c1) if rows[q] != 5][0]
    col[off - c0] = free[-1]
    order = np.argsort(col)
    rows[c0:c1] = np.array(col)[order]
    vals = B.val.copy()
    vals[c0:c1] = vals[c0:c1][order]
    dA.rowidx.copy_(torch.from_numpy(rows.astype(np.int32)).cuda())
    dA.val.copy_(torch.from_numpy(vals).cuda())
    with pytest.raises(diaf.DiafError) as ei:
        diaf.diaf_refactor(ctx, dA, F)
    assert ei.value.code == diaf.DIAF_EINVAL
    F.close()
    say("case value-dependent W pattern")
    A2 = synth.random_lognormal(500, 3)
    dA2 = diaf.DeviceCSC.from_host(A2)
    F2 = diaf.diaf_factor(ctx, dA2, diaf.make_spec(w="A_1hop_topk", w_topk=4, v="diag"), "unit_v")
    with pytest.raises(diaf.DiafError) as ei:
        diaf.diaf_refactor(ctx, dA2, F2)
    assert ei.value.code == diaf.DIAF_EUNSUPPORTED
    F2.close()


def test_refactor_without_graph_matches(ctx):
    """factor_graph = 0: every refactor runs eagerly; same results."""
    import torch
    from paper_1208_3573_amd import diaf
    A = synth.convdiff(12, 3, 9)
    dA = diaf.DeviceCSC.from_host(A)
    spec = diaf.make_spec(w="A2", v="topk_lower", v_count=5)
    F = diaf.diaf_factor(ctx, dA, spec, "unit_v")
    ctx.set_option("factor_graph", 0)
    try:
        for seed in (5, 6):
            dA.val.copy_(torch.from_numpy(_perturbed(A, seed)).cuda())
            diaf.diaf_refactor(ctx, dA, F)
            H = F.to_host()
            Fr = diaf.diaf_factor(ctx, dA, spec, "unit_v")
            Hr = Fr.to_host()
            for key in KEYS:
                assert np.array_equal(np.asarray(H[key]), np.asarray(Hr[key])), key
            Fr.close()
    finally:
        ctx.set_option("factor_graph", 1)
    F.close()
