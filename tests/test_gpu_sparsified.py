"""GPU sparsified powers W pattern (Algorithm 1, Section 4) against the
oracle, bit-exact, factor parity with it, and the error paths."""
import numpy as np
import pytest

import oracle
import synth
from tests._gpu import compare, say

pytestmark = pytest.mark.gpu

PARAMS = [
    dict(k=1, tau_i=0.0),
    dict(k=2, tau_i=0.0),
    dict(k=3, tau_i=0.1),
    dict(k=3, tau_i=0.05, p_i=3, tau_l=0.1, p_l=4),
    dict(k=4, tau_i=0.0, p_i=2, p_l=3),
    dict(k=3, tau_i=0.0, tau_l=0.99, p_l=1),
]

MATS = {
    "convdiff3d_12": lambda: synth.convdiff(12, 3, 7),
    "laplace2d_20": lambda: synth.convdiff(20, 2, 0, beta_max=0.0),  # equal magnitudes: ties
    "random_small": lambda: synth.random_small(500, 4, 3),
    "lognormal_2k": lambda: synth.random_lognormal(2000, 11),
}


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_1208_3573_amd import diaf
    assert torch.cuda.is_available()
    return diaf.Context(0)


def _check(ctx, A, dA, prm):
    from paper_1208_3573_amd import diaf
    cp, ri = diaf.diaf_pattern_build_sparsified(ctx, dA, **prm)
    P = oracle.pattern_sparsified_powers(A, **prm)
    assert np.array_equal(cp.cpu().numpy(), P.colptr)
    assert np.array_equal(ri.cpu().numpy(), P.rowidx)
    return P


@pytest.mark.parametrize("name", list(MATS))
def test_sparsified_patterns_match_oracle(ctx, name):
    from paper_1208_3573_amd import diaf
    A = MATS[name]()
    dA = diaf.DeviceCSC.from_host(A)
    for prm in PARAMS:
        say(f"case {name} n={A.n} {prm}")
        _check(ctx, A, dA, prm)


def test_sparsified_large_tables(ctx):
    """Columns whose power vectors exceed 256 rows take the second, larger
    LDS configuration; results still match bit for bit."""
    from paper_1208_3573_amd import diaf
    A = synth.random_small(3000, 7, 9)
    dA = diaf.DeviceCSC.from_host(A)
    say(f"case random_small n={A.n} k=3 no dropping (large tables)")
    P = _check(ctx, A, dA, dict(k=3, tau_i=0.0))
    assert np.max(np.diff(P.colptr)) > 256


def test_sparsified_empty_and_tiny(ctx):
    from paper_1208_3573_amd import diaf
    for n in (1, 2, 3):
        A = synth.random_small(n, 2, n)
        dA = diaf.DeviceCSC.from_host(A)
        say(f"case tiny n={n}")
        _check(ctx, A, dA, dict(k=3, tau_i=0.0))


@pytest.mark.parametrize("prm,v,l", [(dict(k=2, tau_i=0.0), "topk_lower", 4),
                                     (dict(k=3, tau_i=0.1, p_l=6), "gs_upper", 0),
                                     (dict(k=3, tau_i=0.05, tau_l=0.2), "diag", 0)])
def test_factor_with_sparsified_pattern_matches_oracle(ctx, prm, v, l):
    from paper_1208_3573_amd import diaf
    A = synth.convdiff(12, 3, 7)
    dA = diaf.DeviceCSC.from_host(A)
    J = oracle.pattern_sparsified_powers(A, **prm)
    for mode in ("unit_v", "unit_w"):
        say(f"factor {prm} V {v} mode {mode}")
        F = diaf.diaf_factor(ctx, dA, diaf.make_spec(w="sparsified", v=v, v_count=l,
                                                     sparsify=prm), mode)
        H = F.to_host()
        assert np.array_equal(H["Wcp"], J.colptr) and np.array_equal(H["Wri"], J.rowidx)
        O = oracle.factor(A, J, mode, v, l)
        compare(H, J, O, A, mode)
        F.close()


def test_sparsified_errors(ctx):
    from paper_1208_3573_amd import diaf
    A = synth.random_small(40, 3, 0)
    dA = diaf.DeviceCSC.from_host(A)
    for bad in (dict(k=0), dict(k=9), dict(tau_i=-1.0), dict(tau_l=float("nan")), dict(p_l=-1)):
        say(f"case bad parameters {bad}")
        with pytest.raises(diaf.DiafError) as ei:
            diaf.diaf_pattern_build_sparsified(ctx, dA, **bad)
        assert ei.value.code == diaf.DIAF_EINVAL
        with pytest.raises(diaf.DiafError) as ei:
            diaf.diaf_factor(ctx, dA, diaf.make_spec(w="sparsified", sparsify=bad), "unit_v")
        assert ei.value.code == diaf.DIAF_EINVAL
    say("case complex matrix")
    Ac = synth.random_small(40, 3, 0, complex_=True)
    dAc = diaf.DeviceCSC.from_host(Ac)
    with pytest.raises(diaf.DiafError) as ei:
        diaf.diaf_pattern_build_sparsified(ctx, dAc)
    assert ei.value.code == diaf.DIAF_EUNSUPPORTED
    with pytest.raises(diaf.DiafError) as ei:
        diaf.diaf_factor(ctx, dAc, diaf.make_spec(w="sparsified"), "unit_v")
    assert ei.value.code == diaf.DIAF_EUNSUPPORTED
    say("case zero diagonal")
    Az = synth.random_small(40, 3, 1)
    dpos = [q for q in range(Az.colptr[4], Az.colptr[5]) if Az.rowidx[q] == 4][0]
    Az.val[dpos] = 0.0
    with pytest.raises(diaf.DiafError) as ei:
        diaf.diaf_pattern_build_sparsified(ctx, diaf.DeviceCSC.from_host(Az))
    assert ei.value.code == diaf.DIAF_EINVAL
    say("case power vectors beyond 2048 rows")
    Ab = synth.random_small(6000, 20, 2)
    with pytest.raises(diaf.DiafError) as ei:
        diaf.diaf_pattern_build_sparsified(ctx, diaf.DeviceCSC.from_host(Ab), k=3, tau_i=0.0)
    assert ei.value.code == diaf.DIAF_EUNSUPPORTED
    say("case a column of A longer than 1024")
    n = 1100
    rows = np.concatenate([np.arange(n), np.arange(n)])
    cols = np.concatenate([np.arange(n), np.zeros(n, dtype=np.int64)])
    vals = np.concatenate([np.full(n, 4.0), np.full(n, -1e-3)])
    keep = ~((rows == 0) & (cols == 0) & (np.arange(2 * n) >= n))
    Al = synth._coo_to_csc(n, rows[keep], cols[keep], vals[keep])
    with pytest.raises(diaf.DiafError) as ei:
        diaf.diaf_pattern_build_sparsified(ctx, diaf.DeviceCSC.from_host(Al), k=1)
    assert ei.value.code == diaf.DIAF_EUNSUPPORTED


def test_sparsified_diagonal_matrix(ctx):
    from paper_1208_3573_amd import diaf
    n = 300
    A = synth._coo_to_csc(n, np.arange(n), np.arange(n), np.linspace(1.0, 3.0, n))
    dA = diaf.DeviceCSC.from_host(A)
    say("case diagonal matrix")
    P = _check(ctx, A, dA, dict(k=4, tau_i=0.0))
    assert P.nnz == n
