"""The allocation-free apply (diaf_apply_noalloc) against diaf_apply,
through the C ABI: bit-identical outputs on two calls in a row, the second
with a smaller problem, for a triangular, a diagonal and a block diagonal
V, real and complex; its limits (factors not yet prepared, n beyond the
scratch array) are errors, not faults."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_1208_3573_amd import diaf
    assert torch.cuda.is_available()
    return diaf.Context(0)


def _prepared(ctx, A, **kw):
    import torch
    from paper_1208_3573_amd import diaf
    dA = diaf.DeviceCSC.from_host(A)
    F = diaf.diaf_factor(ctx, dA, diaf.make_spec(**kw), "unit_v")
    dt = dA.torch_dtype
    x0 = torch.zeros(A.n, dtype=dt, device="cuda")
    y0 = torch.zeros_like(x0)
    diaf.diaf_apply(ctx, F, x0, y0)  # builds the row-oriented copies
    return dA, F


def _compare(ctx, F, n, dt, seed):
    import torch
    from paper_1208_3573_amd import diaf
    g = torch.Generator(device="cuda").manual_seed(seed)
    x = torch.randn(n, dtype=torch.float64, device="cuda", generator=g)
    if dt == torch.complex128:
        x = torch.complex(x, torch.randn(n, dtype=torch.float64, device="cuda", generator=g))
    y_ref = torch.full_like(x, float("nan"))
    y = torch.full_like(x, float("nan"))
    diaf.diaf_apply(ctx, F, x, y_ref)
    diaf.diaf_apply_noalloc(ctx, F, x, y)
    torch.cuda.synchronize()
    a = torch.view_as_real(y).cpu().numpy() if y.is_complex() else y.cpu().numpy()
    b = torch.view_as_real(y_ref).cpu().numpy() if y.is_complex() else y_ref.cpu().numpy()
    assert np.all(np.isfinite(b))
    assert np.array_equal(a.view(np.uint64), b.view(np.uint64))


@pytest.mark.parametrize("kind", ["triangular", "diagonal", "block", "complex"])
def test_noalloc_apply_matches_apply(ctx, kind):
    big, small = synth.convdiff(24, 3, 5), synth.convdiff(10, 3, 6)
    if kind == "complex":
        big, small = synth.helmholtz(64, 10.0, 0.5), synth.helmholtz(20, 10.0, 0.5)
    kws = {"triangular": dict(w="A2", v="topk_lower", v_count=5),
           "diagonal": dict(w="A2", v="diag"),
           "complex": dict(w="A2", v="gs_upper")}
    for seed, A in ((1, big), (2, small)):
        kw = kws.get(kind)
        if kind == "block":
            import torch
            kw = dict(w="A2", v="topk_block", v_count=4,
                      v_blocks=torch.arange(0, A.n + 1, 8, dtype=torch.int32, device="cuda"))
        dA, F = _prepared(ctx, A, **kw)
        _compare(ctx, F, A.n, dA.torch_dtype, seed)
        F.close()


def test_noalloc_apply_limits(ctx):
    import torch
    from paper_1208_3573_amd import diaf
    A = synth.convdiff(8, 3, 2)
    dA = diaf.DeviceCSC.from_host(A)
    F = diaf.diaf_factor(ctx, dA, diaf.make_spec(w="A2", v="topk_lower", v_count=5), "unit_v")
    x = torch.ones(A.n, dtype=torch.float64, device="cuda")
    y = torch.zeros_like(x)
    with pytest.raises(diaf.DiafError) as ei:
        diaf.diaf_apply_noalloc(ctx, F, x, y)  # not prepared yet
    assert ei.value.code == diaf.DIAF_EINVAL
    diaf.diaf_apply(ctx, F, x, y)
    diaf.diaf_apply_noalloc(ctx, F, x, y)
    F.close()
    # n beyond the scratch array: a diagonal matrix of 2.2 M rows
    n = 2_200_000
    import scipy.sparse as sp
    D = synth.CSC.from_scipy(sp.diags(np.full(n, 2.0)).tocsc())
    dD = diaf.DeviceCSC.from_host(D)
    F = diaf.diaf_factor(ctx, dD, diaf.make_spec(w="A", v="diag"), "unit_v")
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.zeros_like(x)
    diaf.diaf_apply(ctx, F, x, y)
    with pytest.raises(diaf.DiafError) as ei:
        diaf.diaf_apply_noalloc(ctx, F, x, y)
    assert ei.value.code == diaf.DIAF_EINVAL
    F.close()
