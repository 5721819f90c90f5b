"""GPU parity of the Section 3.1 V rule (the diagonal plus the admissible
rows whose columns of Q_j^* have the largest norms) against the CPU oracle,
through the C ABI, in the small-column and the generic kernels.  Same bars
as the other factor parity tests (identical V patterns, residual and angle
bars)."""
import numpy as np
import pytest

import oracle
import synth
from tests._gpu import compare, oracle_pattern, say

pytestmark = pytest.mark.gpu

CASES = {
    # name: (matrix, W rule, wtopk, V rule, l, generic_only)
    "small_real_lower": (lambda: synth.random_small(300, 3, 5, diag_shift=1.0), "A2", 0,
                         "lev_lower", 4, False),
    "small_complex_upper": (lambda: synth.random_small(300, 3, 6, complex_=True, diag_shift=1.0),
                            "A2", 0, "lev_upper", 4, False),
    "convdiff3d_16": (lambda: synth.convdiff(16, 3, 7), "A2", 0, "lev_lower", 5, False),
    "generic_lognormal_1hop": (lambda: synth.random_lognormal(3000, 11), "A_1hop_topk", 8,
                               "lev_lower", 5, False),
    "generic_only_convdiff": (lambda: synth.convdiff(12, 3, 3), "A2", 0, "lev_upper", 5, True),
}


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_1208_3573_amd import diaf
    assert torch.cuda.is_available()
    return diaf.Context(0)


@pytest.mark.parametrize("name", list(CASES))
def test_leverage_rule_matches_oracle(ctx, name):
    from paper_1208_3573_amd import diaf
    build, w, wtopk, v, l, generic = CASES[name]
    A = build()
    J = oracle_pattern(A, w, wtopk)
    say(f"case {name} n={A.n} generic_only={generic}")
    ctx.set_option("generic_only", 1 if generic else 0)
    try:
        dA = diaf.DeviceCSC.from_host(A)
        F = diaf.diaf_factor(ctx, dA, diaf.make_spec(w=w, w_topk=wtopk, v=v, v_count=l),
                             "unit_v")
        H = F.to_host()
    finally:
        ctx.set_option("generic_only", 0)
    O = oracle.factor(A, J, "unit_v", v, l)
    compare(H, J, O, A, "unit_v")
    F.close()


def test_leverage_rule_with_the_constraint(ctx):
    """The Section 3.2 constraint applies to the rule's triangular V."""
    from paper_1208_3573_amd import diaf
    A = synth.random_small(400, 4, 0)
    J = oracle.pattern_A(A)
    dA = diaf.DeviceCSC.from_host(A)
    F = diaf.diaf_factor(ctx, dA, diaf.make_spec(w="A", v="lev_lower", v_count=5, stab_r=2.0),
                         "unit_v")
    H = F.to_host()
    O = oracle.factor(A, J, "unit_v", "lev_lower", 5, stab_r=2.0)
    compare(H, J, O, A, "unit_v")
    g = np.nonzero(H["flags"] & oracle.STABILIZED)[0]
    assert len(g) >= 1 and np.array_equal(g, np.nonzero(O.flags & oracle.STABILIZED)[0])
    F.close()


def test_leverage_rule_rejects_unit_w(ctx):
    from paper_1208_3573_amd import diaf
    A = synth.random_small(50, 3, 0)
    dA = diaf.DeviceCSC.from_host(A)
    with pytest.raises(diaf.DiafError):
        diaf.diaf_factor(ctx, dA, diaf.make_spec(w="A", v="lev_lower", v_count=3), "unit_w")
