"""The method variants at the full 64^3 size, in the configuration
bench.py --variants times: Algorithm 1 (paper parameters k = 3, tau_i = 0.1)
and Algorithm 2 patterns, block diagonal V on the x-lines of the grid, and
the left variant.  Patterns are compared bit for bit (Algorithm 1 on a sample
of columns the oracle recomputes one by one); factors on sampled columns."""
import numpy as np
import pytest

import oracle
import synth
from tests._gpu import compare, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_1208_3573_amd import diaf
    assert torch.cuda.is_available()
    return diaf.Context(0)


@pytest.fixture(scope="module")
def A64():
    return synth.workload_matrix("convdiff3d_64")


def _sample(n, k, seed):
    rng = np.random.default_rng(seed)
    s = set(rng.choice(n, size=min(k, n), replace=False).tolist())
    s |= {0, 1, 63, 64, 4095, 4096, n // 2, n - 2, n - 1}
    return np.array(sorted(s))


def test_alg1_full_size_sampled(ctx, A64):
    from paper_1208_3573_amd import diaf
    A = A64
    dA = diaf.DeviceCSC.from_host(A)
    prm = dict(k=3, tau_i=0.1, p_i=0, tau_l=0.0, p_l=0)
    say(f"case Algorithm 1 at n={A.n} {prm}")
    cp, ri = diaf.diaf_pattern_build_sparsified(ctx, dA, **prm)
    cp, ri = cp.cpu().numpy(), ri.cpu().numpy()
    assert cp[0] == 0 and np.all(np.diff(cp) >= 1)
    cols = _sample(A.n, 1500, 3)
    ref = oracle.sparsified_powers_columns(A, cols, **prm)
    for j in cols:
        assert np.array_equal(ri[cp[j]:cp[j + 1]], ref[j]), j
    say(f"nnz(W) {cp[-1]}, {len(cols)} columns compared")


def test_alg2_full_size(ctx, A64):
    from paper_1208_3573_amd import diaf
    A = A64
    dA = diaf.DeviceCSC.from_host(A)
    for v0 in ("gs_lower", "diag"):
        say(f"case Algorithm 2 V_0 {v0} at n={A.n}")
        cp, ri = diaf.diaf_pattern_build(ctx, dA, f"alg2_{v0}")
        P = oracle.pattern_alg2(A, v0)
        assert np.array_equal(cp.cpu().numpy(), P.colptr)
        assert np.array_equal(ri.cpu().numpy(), P.rowidx)


@pytest.mark.parametrize("v,l", [("block", 0), ("topk_block", 5)])
def test_block_v_full_size_sampled(ctx, A64, v, l):
    import torch
    from paper_1208_3573_amd import diaf
    A = A64
    st = np.arange(0, A.n + 1, 64, dtype=np.int32)
    dA = diaf.DeviceCSC.from_host(A)
    J = oracle.pattern_A2(A)
    cols = _sample(A.n, 1500, 4)
    for mode in ("unit_v", "unit_w"):
        say(f"case block V {v} l={l} mode {mode} at n={A.n}")
        spec = diaf.make_spec(w="A2", v=v, v_count=l,
                              v_blocks=torch.from_numpy(st).cuda())
        F = diaf.diaf_factor(ctx, dA, spec, mode)
        H = F.to_host()
        if v == "block":
            O = oracle.factor(A, J, mode, "explicit", Vexp=oracle.pattern_vblock(A, st), cols=cols)
        else:
            O = oracle.factor(A, J, mode, "topk_block", l, vblocks=st, cols=cols)
        compare(H, J, O, A, mode, cols=cols)
        F.close()


def test_left_full_size_sampled(ctx, A64):
    from paper_1208_3573_amd import diaf
    import scipy.sparse as sp
    A = A64
    Ah = oracle.conj_transpose(A)
    J = oracle.pattern_A2(Ah)
    dA = diaf.DeviceCSC.from_host(A)
    cols = _sample(A.n, 1500, 5)
    say(f"case left variant at n={A.n}")
    F = diaf.diaf_factor(ctx, dA, diaf.make_spec(w="A2", v="topk_lower", v_count=5, left=True),
                         "unit_v")
    H = F.to_host()
    n = A.n
    back = dict(H)
    for cpk, rik, vak in (("Wcp", "Wri", "Wval"), ("Vcp", "Vri", "Vval")):
        M = sp.csc_matrix((H[vak], H[rik], H[cpk]), shape=(n, n)).conj().T.tocsc()
        M.sort_indices()
        back[cpk], back[rik], back[vak] = (M.indptr.astype(np.int32),
                                           M.indices.astype(np.int32), M.data)
    O = oracle.factor(Ah, J, "unit_v", "topk_lower", 5, cols=cols)
    compare(back, J, O, Ah, "unit_v", cols=cols)
    F.close()
