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
    import torch
    for starts, code, what in ((np.array([0, 20, 39]), diaf.DIAF_EINVAL, "starts not ending at n"),
                               (np.array([0, 20, 20, 40]), diaf.DIAF_EINVAL, "empty block"),
                               (np.array([0, 40]), diaf.DIAF_OK, "one block of 40 rows")):
        say(f"case V_0 blocks: {what}")
        vb = torch.from_numpy(starts.astype(np.int32)).cuda()
        if code == diaf.DIAF_OK:
            diaf.diaf_pattern_build_sparsified(ctx, dA, v0_blocks=vb)
            continue
        with pytest.raises(diaf.DiafError) as ei:
            diaf.diaf_pattern_build_sparsified(ctx, dA, v0_blocks=vb)
        assert ei.value.code == code
    say("case V_0 block of more than 64 rows")
    A2 = synth.random_small(130, 3, 0)
    vb = torch.tensor([0, 65, 130], dtype=torch.int32, device="cuda")
    with pytest.raises(diaf.DiafError) as ei:
        diaf.diaf_pattern_build_sparsified(ctx, diaf.DeviceCSC.from_host(A2), v0_blocks=vb)
    assert ei.value.code == diaf.DIAF_EUNSUPPORTED
    say("case singular V_0 block")
    rows = np.array([0, 1, 0, 1, 2, 3, 2, 3])
    cols = np.array([0, 0, 1, 1, 2, 2, 3, 3])
    vals = np.array([1.0, 1.0, 1.0, 1.0, 2.0, 0.5, 0.5, 2.0])
    As = synth._coo_to_csc(4, rows, cols, vals)
    vb = torch.tensor([0, 2, 4], dtype=torch.int32, device="cuda")
    with pytest.raises(diaf.DiafError) as ei:
        diaf.diaf_pattern_build_sparsified(ctx, diaf.DeviceCSC.from_host(As), v0_blocks=vb)
    assert ei.value.code == diaf.DIAF_EINVAL
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


# ---- complex A, block diagonal V_0 and the final removal --------------------

COMPLEX_MATS = {
    "random_small_complex": lambda: synth.random_small(400, 4, 5, complex_=True),
    "helmholtz_16": lambda: synth.helmholtz(16),
}


@pytest.mark.parametrize("name", list(COMPLEX_MATS))
def test_complex_diagonal_v0_matches_oracle_bit_for_bit(ctx, name):
    """Complex A with the diagonal V_0: the products and the division are
    spelled out alike on both sides, so the patterns agree exactly."""
    from paper_1208_3573_amd import diaf
    A = COMPLEX_MATS[name]()
    dA = diaf.DeviceCSC.from_host(A)
    for prm in PARAMS:
        say(f"case {name} n={A.n} {prm}")
        _check(ctx, A, dA, prm)


def _blocks(n, sizes):
    s = [0]
    q = 0
    while s[-1] < n:
        s.append(min(n, s[-1] + sizes[q % len(sizes)]))
        q += 1
    return np.array(s, dtype=np.int32)


BLOCK_CASES = {
    "convdiff3d_12_xlines": (lambda: synth.convdiff(12, 3, 7), lambda n: np.arange(0, n + 1, 12)),
    "random_small_mixed": (lambda: synth.random_small(500, 4, 3), lambda n: _blocks(n, [5, 7, 3, 8])),
    "random_complex_mixed": (lambda: synth.random_small(400, 4, 5, complex_=True),
                             lambda n: _blocks(n, [6, 4, 9])),
    "helmholtz_16_xlines": (lambda: synth.helmholtz(16), lambda n: np.arange(0, n + 1, 16)),
}
BLOCK_PARAMS = [dict(k=1, tau_i=0.0), dict(k=3, tau_i=0.1),
                dict(k=3, tau_i=0.05, p_i=8, tau_l=0.1, p_l=12)]


def _compare_block(A, cols, got_cp, got_ri, starts, prm, tag, bound=0.01):
    """Columns whose oracle decisions all lie farther than 1e-9 (relative)
    from a dropping boundary must match exactly; the others, where rounding
    of the LU solves can decide, are counted and bounded."""
    ref = oracle.sparsified_powers_columns(A, cols, **prm, v0_blocks=starts, with_margin=True)
    amb = mism = 0
    for j in cols:
        rows, m = ref[int(j)]
        got = got_ri[got_cp[j]:got_cp[j + 1]]
        if m <= 1e-9:
            amb += 1
            continue
        mism += not np.array_equal(got, rows)
        assert np.array_equal(got, rows), (tag, int(j), m)
    say(f"{tag}: {len(cols)} columns, {amb} within rounding of a dropping boundary")
    assert amb <= bound * len(cols)


@pytest.mark.parametrize("name", list(BLOCK_CASES))
def test_block_v0_patterns_match_oracle(ctx, name):
    import torch
    from paper_1208_3573_amd import diaf
    mk, blk = BLOCK_CASES[name]
    A = mk()
    starts = blk(A.n).astype(np.int32)
    vb = torch.from_numpy(starts).cuda()
    dA = diaf.DeviceCSC.from_host(A)
    for prm in BLOCK_PARAMS:
        say(f"case {name} n={A.n} blocks={len(starts) - 1} {prm}")
        cp, ri = diaf.diaf_pattern_build_sparsified(ctx, dA, **prm, v0_blocks=vb)
        cp, ri = cp.cpu().numpy(), ri.cpu().numpy()
        _compare_block(A, range(A.n), cp, ri, starts, prm, f"{name} {prm}")
        # the removal: inside its block a column keeps its diagonal only
        lo = np.repeat(starts[:-1], np.diff(starts))
        hi = np.repeat(starts[1:], np.diff(starts))
        col = np.repeat(np.arange(A.n), np.diff(cp))
        inside = (ri >= lo[col]) & (ri < hi[col])
        assert np.array_equal(ri[inside], col[inside])


def test_block_v0_full_size_64(ctx):
    """The 64^3 workload with V_0 block diagonal on the x-lines (64 rows),
    the paper's parameters (k = 3, tau_i = 0.1): 300 sampled columns (block
    ends and random) against the oracle."""
    import torch
    from paper_1208_3573_amd import diaf
    A = synth.workload_matrix("convdiff3d_64")
    starts = np.arange(0, A.n + 1, 64, dtype=np.int32)
    dA = diaf.DeviceCSC.from_host(A)
    prm = dict(k=3, tau_i=0.1)
    say("case convdiff3d_64 x-line blocks k=3 tau_i=0.1")
    cp, ri = diaf.diaf_pattern_build_sparsified(ctx, dA, **prm,
                                                v0_blocks=torch.from_numpy(starts).cuda())
    cp, ri = cp.cpu().numpy(), ri.cpu().numpy()
    rng = np.random.default_rng(5)
    cols = np.unique(np.concatenate([rng.choice(A.n, 250, replace=False),
                                     [0, 63, 64, 4095, 4096, A.n - 64, A.n - 1]]))
    _compare_block(A, cols, cp, ri, starts, prm, "convdiff3d_64")
    say(f"nnz(W) {len(ri)} (mean |J_j| {len(ri) / A.n:.1f})")


def test_factor_with_block_v0_pattern_matches_oracle(ctx):
    import torch
    from paper_1208_3573_amd import diaf
    A = synth.convdiff(10, 3, 2)
    starts = np.arange(0, A.n + 1, 10, dtype=np.int32)
    vb = torch.from_numpy(starts).cuda()
    prm = dict(k=2, tau_i=0.1)
    dA = diaf.DeviceCSC.from_host(A)
    ref = oracle.sparsified_powers_columns(A, range(A.n), **prm, v0_blocks=starts,
                                           with_margin=True)
    assert min(m for _, m in ref.values()) > 1e-9
    J = oracle.pattern_sparsified_powers(A, **prm, v0_blocks=starts)
    for mode in ("unit_v", "unit_w"):
        say(f"factor block V_0 {prm} mode {mode}")
        F = diaf.diaf_factor(ctx, dA, diaf.make_spec(w="sparsified", v="topk_lower", v_count=4,
                                                     sparsify=dict(prm, v0_blocks=vb)), mode)
        H = F.to_host()
        assert np.array_equal(H["Wcp"], J.colptr) and np.array_equal(H["Wri"], J.rowidx)
        O = oracle.factor(A, J, mode, "topk_lower", 4)
        compare(H, J, O, A, mode)
        F.close()
