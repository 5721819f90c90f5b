"""GPU parity of the constrained computation of Section 3.2 (unit-norm v,
triangular V, v_jj := stab_r where |v_jj| < stab_tol ||v_j||) against the
CPU oracle, through the C ABI, in the small-column kernel and in the generic
kernel.

Bars: the same columns constrained on both sides; the usual residual and
subspace-angle bars of the parity tests; and, since v_j then has a fixed
scale and phase (v_jj = stab_r, the phase of the rest fixed by the rule),
v_j entrywise within 1e-8 ||v_j|| and w_j within 1e-7 ||w_j||.
"""
import numpy as np
import pytest

import oracle
import synth
from tests._gpu import angle_excluded, compare, oracle_pattern, say

pytestmark = pytest.mark.gpu

R = 2.0

CASES = {
    # name: (matrix, W rule, V rule, l, generic_only)
    "small_kernel_A_lower": (lambda: synth.random_small(400, 4, 0), "A", "topk_lower", 5, False),
    "small_kernel_A2_upper": (lambda: synth.random_small(400, 4, 1), "A2", "topk_upper", 4, False),
    "small_kernel_gs_upper": (lambda: synth.random_small(400, 4, 2), "A2", "gs_upper", 0, False),
    "small_kernel_complex": (lambda: synth.random_small(400, 4, 0, complex_=True), "A2",
                             "topk_lower", 5, False),
    "generic_kernel_A2_k73": (lambda: synth.random_small(400, 8, 0), "A2", "topk_lower", 5, False),
    "generic_only_complex": (lambda: synth.random_small(400, 4, 3, complex_=True), "A2",
                             "topk_upper", 4, True),
    "generic_only_real": (lambda: synth.random_small(400, 4, 2), "A", "topk_lower", 5, True),
}


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_1208_3573_amd import diaf
    assert torch.cuda.is_available()
    return diaf.Context(0)


@pytest.mark.parametrize("name", list(CASES))
def test_stabilized_columns_match_oracle(ctx, name):
    from paper_1208_3573_amd import diaf
    build, w, v, l, generic = CASES[name]
    A = build()
    J = oracle_pattern(A, w)
    say(f"case {name} n={A.n} generic_only={generic}")
    ctx.set_option("generic_only", 1 if generic else 0)
    try:
        dA = diaf.DeviceCSC.from_host(A)
        F = diaf.diaf_factor(ctx, dA, diaf.make_spec(w=w, v=v, v_count=l, stab_r=R), "unit_v")
        H = F.to_host()
        st = F.stats()
    finally:
        ctx.set_option("generic_only", 0)
    O = oracle.factor(A, J, "unit_v", v, l, stab_r=R)
    compare(H, J, O, A, "unit_v")
    g_st = np.nonzero(H["flags"] & oracle.STABILIZED)[0]
    o_st = np.nonzero(O.flags & oracle.STABILIZED)[0]
    say(f"  constrained columns: gpu {len(g_st)} oracle {len(o_st)}, stats {st.count_stabilized}")
    assert len(o_st) >= 3
    assert np.array_equal(g_st, o_st)
    assert st.count_stabilized == len(o_st)
    assert np.array_equal(np.nonzero(H["flags"] & oracle.SMALL_DIAG)[0],
                          np.nonzero(O.flags & oracle.SMALL_DIAG)[0])
    worst_v = worst_w = 0.0
    for j in o_st:
        if angle_excluded(O.flags[j], "unit_v"):
            continue
        gv = H["Vval"][H["Vcp"][j]:H["Vcp"][j + 1]]
        ov = O.Vvals_pad[j, :O.lcount[j]]
        dv = np.max(np.abs(gv - ov)) / np.linalg.norm(ov)
        sl = slice(J.colptr[j], J.colptr[j + 1])
        dw = np.linalg.norm(H["Wval"][sl] - O.Wval[sl]) / np.linalg.norm(O.Wval[sl])
        worst_v, worst_w = max(worst_v, dv), max(worst_w, dw)
        assert dv <= 1e-8, (j, dv)
        assert dw <= 1e-7, (j, dw)
    say(f"  worst v {worst_v:.2e} worst w {worst_w:.2e}")
    F.close()


def test_stabilization_off_leaves_factors_unchanged(ctx):
    """stab_r = 0 gives bit-identical factors to a spec without it, and the
    constrained run differs only in the constrained columns."""
    from paper_1208_3573_amd import diaf
    A = synth.random_small(400, 4, 0)
    dA = diaf.DeviceCSC.from_host(A)
    H0 = diaf.diaf_factor(ctx, dA, diaf.make_spec(w="A", v="topk_lower", v_count=5),
                          "unit_v").to_host()
    H1 = diaf.diaf_factor(ctx, dA, diaf.make_spec(w="A", v="topk_lower", v_count=5, stab_r=R),
                          "unit_v").to_host()
    st = np.nonzero(H1["flags"] & oracle.STABILIZED)[0]
    assert len(st) >= 3
    other = np.setdiff1d(np.arange(A.n), st)
    for j in other:
        a = slice(H0["Vcp"][j], H0["Vcp"][j + 1])
        b = slice(H1["Vcp"][j], H1["Vcp"][j + 1])
        assert np.array_equal(H0["Vval"][a], H1["Vval"][b])
    assert np.array_equal(np.nonzero(H0["flags"] & oracle.SMALL_DIAG)[0], st)


def test_stabilization_rejects_bad_parameters(ctx):
    from paper_1208_3573_amd import diaf
    A = synth.random_small(50, 3, 0)
    dA = diaf.DeviceCSC.from_host(A)
    for r, tol in ((-1.0, 1e-2), (float("nan"), 1e-2), (2.0, -1.0), (2.0, float("inf"))):
        with pytest.raises(diaf.DiafError):
            diaf.diaf_factor(ctx, dA, diaf.make_spec(w="A", v="diag", stab_r=r, stab_tol=tol),
                             "unit_v")
