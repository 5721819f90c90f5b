"""GPU Algorithm 2 W patterns (Section 4) against the oracle, bit-exact, and
factor parity with them."""
import numpy as np
import pytest

import oracle
import synth
from tests._gpu import compare, say

pytestmark = pytest.mark.gpu

MATS = {
    "convdiff3d_16": lambda: synth.convdiff(16, 3, 7),
    "random_small": lambda: synth.random_small(500, 4, 3),
    "random_small_c": lambda: synth.random_small(400, 3, 6, complex_=True),
    "lognormal_3k": lambda: synth.random_lognormal(3000, 11),
}


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_1208_3573_amd import diaf
    assert torch.cuda.is_available()
    return diaf.Context(0)


@pytest.mark.parametrize("name", list(MATS))
def test_alg2_patterns_match_oracle(ctx, name):
    from paper_1208_3573_amd import diaf
    A = MATS[name]()
    dA = diaf.DeviceCSC.from_host(A)
    for v0 in ("diag", "gs_upper", "gs_lower"):
        say(f"case {name} V_0 {v0} n={A.n}")
        cp, ri = diaf.diaf_pattern_build(ctx, dA, f"alg2_{v0}")
        P = oracle.pattern_alg2(A, v0)
        assert np.array_equal(cp.cpu().numpy(), P.colptr)
        assert np.array_equal(ri.cpu().numpy(), P.rowidx)


@pytest.mark.parametrize("v0,v,l", [("gs_upper", "topk_upper", 4), ("gs_lower", "topk_lower", 5),
                                    ("diag", "diag", 0)])
def test_factor_with_alg2_pattern_matches_oracle(ctx, v0, v, l):
    from paper_1208_3573_amd import diaf
    A = synth.convdiff(16, 3, 7)
    dA = diaf.DeviceCSC.from_host(A)
    J = oracle.pattern_alg2(A, v0)
    for mode in ("unit_v", "unit_w"):
        say(f"V_0 {v0} V {v} mode {mode}")
        F = diaf.diaf_factor(ctx, dA, diaf.make_spec(w=f"alg2_{v0}", v=v, v_count=l), mode)
        H = F.to_host()
        O = oracle.factor(A, J, mode, v, l)
        compare(H, J, O, A, mode)
        F.close()


def test_pattern_build_rejects_unknown_kind(ctx):
    from paper_1208_3573_amd import diaf
    A = synth.random_small(30, 3, 0)
    dA = diaf.DeviceCSC.from_host(A)
    with pytest.raises(diaf.DiafError):
        ctx.check(ctx.lib.diaf_pattern_build(ctx.h, __import__("ctypes").byref(dA.desc), 99, 0,
                                             None, None, None))
