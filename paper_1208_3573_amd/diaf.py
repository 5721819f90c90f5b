"""Python binding of libdiaf (include/diaf.h): ctypes marshalling only.

Every numerical step runs in the HIP library; PyTorch provides device memory
(tensors whose data pointers are passed through) and the HIP stream.  The
binding raises if the library was not built: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_double, c_float, c_int, c_int32, c_int64, c_size_t, c_uint32, c_void_p

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdiaf.so")

# ---- enums / flags (mirrors of include/diaf.h) ----
DIAF_OK, DIAF_EINVAL, DIAF_ENOMEM, DIAF_EDEVICE, DIAF_EUNSUPPORTED, DIAF_ESINGULAR, \
    DIAF_ENOCONV, DIAF_EBREAKDOWN = range(8)
STATUS_NAMES = ["OK", "EINVAL", "ENOMEM", "EDEVICE", "EUNSUPPORTED", "ESINGULAR", "ENOCONV",
                "EBREAKDOWN"]
DIAF_F64, DIAF_C128 = 0, 1
DIAF_UNIT_V, DIAF_UNIT_W = 0, 1
DIAF_W_A, DIAF_W_A2, DIAF_W_A_1HOP_TOPK, DIAF_W_EXPLICIT, DIAF_W_LEARNED, DIAF_W_ALG2_DIAG, \
    DIAF_W_ALG2_GS_UPPER, DIAF_W_ALG2_GS_LOWER, DIAF_W_SPARSIFIED = range(9)
DIAF_V_EXPLICIT, DIAF_V_DIAG, DIAF_V_GS_UPPER, DIAF_V_GS_LOWER, DIAF_V_TOPK_UPPER, \
    DIAF_V_TOPK_LOWER, DIAF_V_LEV_UPPER, DIAF_V_LEV_LOWER, DIAF_V_BLOCK, \
    DIAF_V_TOPK_BLOCK = range(10)
FLAG_RANK_DEFICIENT, FLAG_GAP_DEGENERATE, FLAG_SMALL_DIAG, FLAG_FELL_BACK, FLAG_TIE_EDGE, \
    FLAG_STABILIZED, FLAG_NO_DIAG_ROW, FLAG_NULL_CHOICE = 1, 2, 4, 8, 16, 32, 64, 128
MLP_NFEAT, MLP_HIDDEN = 16, 64
MLP_NPARAM = 64 * 16 + 64 + 64 * 64 + 64 + 64 + 1


class diaf_csc(ctypes.Structure):
    _fields_ = [("n", c_int64), ("nnz", c_int64), ("colptr", c_void_p), ("rowidx", c_void_p),
                ("val", c_void_p), ("dtype", c_int32)]


class diaf_pattern(ctypes.Structure):
    _fields_ = [("n", c_int64), ("nnz", c_int64), ("colptr", c_void_p), ("rowidx", c_void_p)]


class diaf_sparsify(ctypes.Structure):
    _fields_ = [("k", c_int32), ("p_i", c_int32), ("p_l", c_int32), ("v0_nblocks", c_int32),
                ("tau_i", c_double), ("tau_l", c_double), ("v0_blocks", c_void_p)]


class diaf_spec(ctypes.Structure):
    _fields_ = [("w_kind", c_int32), ("w_topk", c_int32), ("w_explicit", POINTER(diaf_pattern)),
                ("model", c_void_p), ("gate_tau", c_double), ("v_kind", c_int32),
                ("v_count", c_int32), ("v_explicit", POINTER(diaf_pattern)),
                ("gram_fp32", c_int32), ("gate_dom", c_double), ("stab_r", c_double),
                ("stab_tol", c_double), ("sparsify", diaf_sparsify), ("v_blocks", c_void_p),
                ("v_nblocks", c_int32), ("left", c_int32)]


class diaf_view(ctypes.Structure):
    _fields_ = [("n", c_int64), ("nnz_w", c_int64), ("nnz_v", c_int64), ("dtype", c_int32),
                ("vtri", c_int32), ("Wcp", c_void_p), ("Wri", c_void_p), ("Wval", c_void_p),
                ("Vcp", c_void_p), ("Vri", c_void_p), ("Vval", c_void_p), ("r", c_void_p),
                ("flags", c_void_p), ("lcount", c_void_p)]


class diaf_stats(ctypes.Structure):
    _fields_ = [("n", c_int64), ("nnz_w", c_int64), ("nnz_v", c_int64), ("kmax", c_int32),
                ("mmax", c_int32), ("nbuckets", c_int32), ("count_rank_deficient", c_int32),
                ("count_gap_degenerate", c_int32), ("count_small_diag", c_int32),
                ("count_tie_edge", c_int32), ("count_fell_back", c_int32),
                ("count_no_diag", c_int32), ("v_levels", c_int32),
                ("count_zero_pivot", c_int32), ("factor_launches", c_int32),
                ("count_deferred", c_int32), ("nrm", c_double),
                ("ms_pattern", c_double), ("ms_factor", c_double), ("ms_assemble", c_double),
                ("ms_factor_kernels", c_double), ("count_stabilized", c_int32),
                ("count_null_choice", c_int32), ("ms_small_kernel", c_double),
                ("ms_generic_class", c_double * 8), ("cols_small", c_int32),
                ("launches_small", c_int32), ("cols_generic_class", c_int32 * 8),
                ("launches_generic_class", c_int32 * 8), ("occ_small", c_double),
                ("occ_generic_class", c_double * 8), ("ms_mid_kernel", c_double),
                ("cols_mid", c_int32), ("launches_mid", c_int32), ("occ_mid", c_double),
                ("class_kcap", c_int32 * 8), ("class_tcap", c_int32 * 8)]


class diaf_solve_info(ctypes.Structure):
    _fields_ = [("iters", c_int32), ("flag", c_int32), ("relres", c_double),
                ("relres_true", c_double), ("ms", c_double)]


_SIGS = {
    "diaf_ctx_create": (c_int, [POINTER(c_void_p), c_int, c_void_p]),
    "diaf_ctx_destroy": (None, [c_void_p]),
    "diaf_last_error": (ctypes.c_char_p, [c_void_p]),
    "diaf_ctx_set_option": (c_int, [c_void_p, ctypes.c_char_p, c_int64]),
    "diaf_ctx_get_option": (c_int, [c_void_p, ctypes.c_char_p, POINTER(c_int64)]),
    "diaf_autotune": (c_int, [c_void_p, POINTER(diaf_csc), POINTER(diaf_spec), c_int32]),
    "diaf_autotune_cached": (c_int, [c_void_p, POINTER(diaf_csc), POINTER(diaf_spec), c_int32,
                                     ctypes.c_char_p, POINTER(c_int32)]),
    "diaf_refactor": (c_int, [c_void_p, POINTER(diaf_csc), c_void_p]),
    "diaf_copy": (c_int, [c_void_p, c_void_p, c_void_p, c_size_t]),
    "diaf_pattern_build": (c_int, [c_void_p, POINTER(diaf_csc), c_int32, c_int32, c_void_p,
                                   c_void_p, POINTER(c_int64)]),
    "diaf_pattern_build_sparsified": (c_int, [c_void_p, POINTER(diaf_csc), POINTER(diaf_sparsify),
                                              c_void_p, c_void_p, POINTER(c_int64)]),
    "diaf_factor": (c_int, [c_void_p, POINTER(diaf_csc), POINTER(diaf_spec), c_int32,
                            POINTER(c_void_p)]),
    "diaf_factors_view": (c_int, [c_void_p, POINTER(diaf_view)]),
    "diaf_factors_stats": (c_int, [c_void_p, POINTER(diaf_stats)]),
    "diaf_factors_levels": (c_int, [c_void_p, c_void_p, POINTER(c_int32)]),
    "diaf_factors_destroy": (None, [c_void_p]),
    "diaf_apply": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "diaf_apply_noalloc": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "diaf_solve": (c_int, [c_void_p, POINTER(diaf_csc), c_void_p, c_void_p, c_void_p, c_double,
                           c_int32, POINTER(diaf_solve_info)]),
    "diaf_model_create": (c_int, [c_void_p, c_void_p, POINTER(c_void_p)]),
    "diaf_model_get_params": (c_int, [c_void_p, c_void_p, c_void_p]),
    "diaf_model_destroy": (None, [c_void_p]),
    "diaf_features": (c_int, [c_void_p, POINTER(diaf_csc), POINTER(diaf_pattern), c_void_p]),
    "diaf_labels": (c_int, [c_void_p, POINTER(diaf_csc), c_void_p, c_double, c_void_p]),
    "diaf_mlp_forward": (c_int, [c_void_p, c_void_p, c_void_p, c_int64, c_void_p]),
    "diaf_mlp_loss_grad": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_int64, c_void_p,
                                   POINTER(c_double)]),
    "diaf_mlp_train_step": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_int64, c_float,
                                    POINTER(c_double)]),
}

EXPORTED = tuple(_SIGS)

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libdiaf.so (raises if it is missing or lacks a symbol)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libdiaf.so not built ({path}); run __graft_entry__.build() or "
                           "python -m paper_1208_3573_amd.build")
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIGS.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


class DiafError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES[code] if 0 <= code < 8 else code}: {msg}")
        self.code = code


# ---------------------------------------------------------------------------
# Thin object layer over the handles (marshalling of torch tensors).
# ---------------------------------------------------------------------------

def _torch():
    import torch
    return torch


class Context:
    """A diaf_ctx on cuda:device ordered on torch's current stream."""

    def __init__(self, device: int = 0, stream=None):
        torch = _torch()
        self.lib = load_library()
        self.device = device
        if stream is None:
            stream = torch.cuda.current_stream(device).cuda_stream
        self.h = c_void_p()
        rc = self.lib.diaf_ctx_create(ctypes.byref(self.h), device, c_void_p(stream))
        if rc != DIAF_OK:
            raise DiafError(rc, "diaf_ctx_create failed")

    def check(self, rc):
        if rc != DIAF_OK:
            raise DiafError(rc, self.lib.diaf_last_error(self.h).decode())
        return rc

    def set_option(self, key: str, value: int):
        self.check(self.lib.diaf_ctx_set_option(self.h, key.encode(), int(value)))

    def get_option(self, key: str) -> int:
        v = c_int64()
        self.check(self.lib.diaf_ctx_get_option(self.h, key.encode(), ctypes.byref(v)))
        return int(v.value)

    def copy(self, dst_ptr: int, src_ptr: int, nbytes: int):
        self.check(self.lib.diaf_copy(self.h, c_void_p(dst_ptr), c_void_p(src_ptr), nbytes))

    def close(self):
        if self.h:
            self.lib.diaf_ctx_destroy(self.h)
            self.h = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class DeviceCSC:
    """A CSC matrix resident on the GPU (torch tensors) and its descriptor."""

    def __init__(self, n, colptr, rowidx, val):
        torch = _torch()
        self.n = int(n)
        self.colptr = colptr
        self.rowidx = rowidx
        self.val = val
        self.dtype = DIAF_C128 if val.dtype == torch.complex128 else DIAF_F64
        self.desc = diaf_csc(self.n, int(rowidx.numel()), colptr.data_ptr(), rowidx.data_ptr(),
                             val.data_ptr(), self.dtype)

    @staticmethod
    def from_host(A, device="cuda"):
        torch = _torch()
        cp = torch.from_numpy(np.ascontiguousarray(A.colptr, dtype=np.int32)).to(device)
        ri = torch.from_numpy(np.ascontiguousarray(A.rowidx, dtype=np.int32)).to(device)
        v = torch.from_numpy(np.ascontiguousarray(A.val)).to(device)
        return DeviceCSC(A.n, cp, ri, v)

    @property
    def torch_dtype(self):
        return self.val.dtype


class DevicePattern:
    def __init__(self, n, colptr, rowidx):
        self.n = int(n)
        self.colptr = colptr
        self.rowidx = rowidx
        self.desc = diaf_pattern(self.n, int(rowidx.numel()), colptr.data_ptr(),
                                 rowidx.data_ptr() if rowidx.numel() else 0)

    @staticmethod
    def from_host(colptr, rowidx, device="cuda"):
        torch = _torch()
        cp = torch.from_numpy(np.ascontiguousarray(colptr, dtype=np.int32)).to(device)
        ri = torch.from_numpy(np.ascontiguousarray(rowidx, dtype=np.int32)).to(device)
        return DevicePattern(len(colptr) - 1, cp, ri)


W_KINDS = {"A": DIAF_W_A, "A2": DIAF_W_A2, "A_1hop_topk": DIAF_W_A_1HOP_TOPK,
           "explicit": DIAF_W_EXPLICIT, "learned": DIAF_W_LEARNED, "alg2_diag": DIAF_W_ALG2_DIAG,
           "alg2_gs_upper": DIAF_W_ALG2_GS_UPPER, "alg2_gs_lower": DIAF_W_ALG2_GS_LOWER,
           "sparsified": DIAF_W_SPARSIFIED}
V_KINDS = {"explicit": DIAF_V_EXPLICIT, "diag": DIAF_V_DIAG, "gs_upper": DIAF_V_GS_UPPER,
           "gs_lower": DIAF_V_GS_LOWER, "topk_upper": DIAF_V_TOPK_UPPER,
           "topk_lower": DIAF_V_TOPK_LOWER, "lev_upper": DIAF_V_LEV_UPPER,
           "lev_lower": DIAF_V_LEV_LOWER, "block": DIAF_V_BLOCK,
           "topk_block": DIAF_V_TOPK_BLOCK}
MODES = {"unit_v": DIAF_UNIT_V, "unit_w": DIAF_UNIT_W}


def make_spec(w="A", v="diag", v_count=0, w_topk=0, w_explicit: DevicePattern | None = None,
              v_explicit: DevicePattern | None = None, model=None, gate_tau=float("inf"),
              gram_fp32=False, gate_dom=0.0, stab_r=0.0, stab_tol=1e-2, sparsify=None,
              v_blocks=None, left=False):
    """sparsify: dict of k, tau_i, p_i, tau_l, p_l for w="sparsified"
    (defaults k=3, tau_i=0.1, no other dropping).  v_blocks: int32 device
    tensor of block starts (0 .. n) for v="block" / "topk_block".  left: the
    left variant W A ~ V, M = V^{-1} W."""
    spec = diaf_spec()
    spec.w_kind = W_KINDS[w]
    spec.w_topk = w_topk
    spec.w_explicit = ctypes.pointer(w_explicit.desc) if w_explicit is not None else None
    spec.model = model.h if model is not None else None
    spec.gate_tau = gate_tau
    spec.v_kind = V_KINDS[v]
    spec.v_count = v_count
    spec.v_explicit = ctypes.pointer(v_explicit.desc) if v_explicit is not None else None
    spec.gram_fp32 = int(bool(gram_fp32))
    spec.gate_dom = gate_dom
    spec.stab_r = stab_r
    spec.stab_tol = stab_tol
    spec.sparsify = make_sparsify(**(sparsify or {}))
    spec.left = int(bool(left))
    if v_blocks is not None:
        assert v_blocks.dtype == _torch().int32 and v_blocks.is_cuda
        spec.v_blocks = c_void_p(v_blocks.data_ptr())
        spec.v_nblocks = v_blocks.numel() - 1
    spec._keep = (w_explicit, v_explicit, model, v_blocks, (sparsify or {}).get("v0_blocks"))
    return spec


class Factors:
    """Owns a diaf_factors handle."""

    def __init__(self, ctx: Context, h: c_void_p, A: DeviceCSC):
        self.ctx = ctx
        self.h = h
        self.A = A

    def view(self) -> diaf_view:
        v = diaf_view()
        self.ctx.check(self.ctx.lib.diaf_factors_view(self.h, ctypes.byref(v)))
        return v

    def stats(self) -> diaf_stats:
        s = diaf_stats()
        self.ctx.check(self.ctx.lib.diaf_factors_stats(self.h, ctypes.byref(s)))
        return s

    def levels(self) -> int:
        """Dependency depth of the V solve (diaf_factors_levels)."""
        out = c_int32(0)
        self.ctx.check(self.ctx.lib.diaf_factors_levels(self.ctx.h, self.h, ctypes.byref(out)))
        return int(out.value)

    def to_host(self):
        """Copy W, V, residuals, flags and l_j to host numpy arrays."""
        v = self.view()
        n = v.n
        cdt = np.complex128 if v.dtype == DIAF_C128 else np.float64

        def get(ptr, count, dt):
            out = np.empty(count, dtype=dt)
            if count:
                self.ctx.copy(out.ctypes.data, ptr, out.nbytes)
            return out

        return dict(
            n=n, vtri=v.vtri,
            Wcp=get(v.Wcp, n + 1, np.int32), Wri=get(v.Wri, v.nnz_w, np.int32),
            Wval=get(v.Wval, v.nnz_w, cdt),
            Vcp=get(v.Vcp, n + 1, np.int32), Vri=get(v.Vri, v.nnz_v, np.int32),
            Vval=get(v.Vval, v.nnz_v, cdt),
            r=get(v.r, n, np.float64), flags=get(v.flags, n, np.uint32),
            lcount=get(v.lcount, n, np.int32),
        )

    def close(self):
        if self.h:
            self.ctx.lib.diaf_factors_destroy(self.h)
            self.h = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def diaf_factor(ctx: Context, A: DeviceCSC, spec: diaf_spec, mode) -> Factors:
    h = c_void_p()
    m = MODES[mode] if isinstance(mode, str) else int(mode)
    ctx.check(ctx.lib.diaf_factor(ctx.h, ctypes.byref(A.desc), ctypes.byref(spec), m,
                                  ctypes.byref(h)))
    return Factors(ctx, h, A)


TUNE_KEYS = ("small_grid", "generic_nt", "class_table", "trsv_waves", "graph", "solve_batch",
             "trsv_backoff")


def diaf_autotune(ctx: Context, A: DeviceCSC, spec: diaf_spec, mode, cache: str | None = None
                  ) -> dict:
    """Tune the context's launch shapes on this problem; returns the choices.
    With `cache` (a file path), a stored choice for this device architecture
    and problem shape is applied instead, and a new one is stored
    (``from_cache`` in the result tells which)."""
    m = MODES[mode] if isinstance(mode, str) else int(mode)
    out = {}
    if cache is None:
        ctx.check(ctx.lib.diaf_autotune(ctx.h, ctypes.byref(A.desc), ctypes.byref(spec), m))
    else:
        hit = c_int32(0)
        ctx.check(ctx.lib.diaf_autotune_cached(ctx.h, ctypes.byref(A.desc), ctypes.byref(spec), m,
                                               os.fsencode(cache), ctypes.byref(hit)))
        out["from_cache"] = bool(hit.value)
    return {k: ctx.get_option(k) for k in TUNE_KEYS} | out


def diaf_refactor(ctx: Context, A: DeviceCSC, F: Factors):
    """Refactor F in place after new values were written into A's value
    buffer (same pattern, same buffers)."""
    ctx.check(ctx.lib.diaf_refactor(ctx.h, ctypes.byref(A.desc), F.h))
    return F


def diaf_apply(ctx: Context, F: Factors, x, y):
    ctx.check(ctx.lib.diaf_apply(ctx.h, F.h, c_void_p(x.data_ptr()), c_void_p(y.data_ptr())))


def diaf_apply_noalloc(ctx: Context, F: Factors, x, y):
    ctx.check(ctx.lib.diaf_apply_noalloc(ctx.h, F.h, c_void_p(x.data_ptr()),
                                         c_void_p(y.data_ptr())))


def diaf_solve(ctx: Context, A: DeviceCSC, F: Factors | None, b, x, rtol=1e-8, maxit=1000,
               raise_on_noconv=False) -> diaf_solve_info:
    info = diaf_solve_info()
    rc = ctx.lib.diaf_solve(ctx.h, ctypes.byref(A.desc), F.h if F is not None else None,
                            c_void_p(b.data_ptr()), c_void_p(x.data_ptr()), rtol, maxit,
                            ctypes.byref(info))
    if rc in (DIAF_ENOCONV, DIAF_EBREAKDOWN, DIAF_ESINGULAR) and not raise_on_noconv:
        return info
    ctx.check(rc)
    return info


def make_sparsify(k=3, tau_i=0.1, p_i=0, tau_l=0.0, p_l=0, v0_blocks=None) -> diaf_sparsify:
    """v0_blocks: None (V_0 diagonal) or an int32 device tensor of block
    starts 0 .. n (V_0 block diagonal); the caller keeps it alive."""
    sp = diaf_sparsify()
    sp.k, sp.p_i, sp.p_l = k, p_i, p_l
    sp.tau_i, sp.tau_l = tau_i, tau_l
    sp.v0_nblocks, sp.v0_blocks = 0, None
    if v0_blocks is not None:
        assert v0_blocks.dtype == _torch().int32 and v0_blocks.is_cuda
        sp.v0_nblocks = v0_blocks.numel() - 1
        sp.v0_blocks = c_void_p(v0_blocks.data_ptr())
    return sp


def diaf_pattern_build_sparsified(ctx: Context, A: DeviceCSC, k=3, tau_i=0.1, p_i=0, tau_l=0.0,
                                  p_l=0, v0_blocks=None):
    """Sparsified powers W pattern (Algorithm 1) on the device; returns
    (colptr, rowidx) tensors."""
    torch = _torch()
    sp = make_sparsify(k, tau_i, p_i, tau_l, p_l, v0_blocks)
    cp = torch.empty(A.n + 1, dtype=torch.int32, device=A.colptr.device)
    nnz = c_int64()
    ctx.check(ctx.lib.diaf_pattern_build_sparsified(ctx.h, ctypes.byref(A.desc), ctypes.byref(sp),
                                                    c_void_p(cp.data_ptr()), None,
                                                    ctypes.byref(nnz)))
    ri = torch.empty(max(1, nnz.value), dtype=torch.int32, device=A.colptr.device)
    ctx.check(ctx.lib.diaf_pattern_build_sparsified(ctx.h, ctypes.byref(A.desc), ctypes.byref(sp),
                                                    c_void_p(cp.data_ptr()),
                                                    c_void_p(ri.data_ptr()), ctypes.byref(nnz)))
    return cp, ri[: nnz.value]


def diaf_pattern_build(ctx: Context, A: DeviceCSC, w_kind: str, w_topk: int = 0):
    """Build a W pattern on the device; returns (colptr, rowidx) tensors."""
    torch = _torch()
    cp = torch.empty(A.n + 1, dtype=torch.int32, device=A.colptr.device)
    nnz = c_int64()
    ctx.check(ctx.lib.diaf_pattern_build(ctx.h, ctypes.byref(A.desc), W_KINDS[w_kind], w_topk,
                                         c_void_p(cp.data_ptr()), None, ctypes.byref(nnz)))
    ri = torch.empty(max(1, nnz.value), dtype=torch.int32, device=A.colptr.device)
    ctx.check(ctx.lib.diaf_pattern_build(ctx.h, ctypes.byref(A.desc), W_KINDS[w_kind], w_topk,
                                         c_void_p(cp.data_ptr()), c_void_p(ri.data_ptr()),
                                         ctypes.byref(nnz)))
    return cp, ri[: nnz.value]


class Model:
    """A learned W-pattern proposer (diaf_model)."""

    def __init__(self, ctx: Context, params: np.ndarray):
        p = np.ascontiguousarray(params, dtype=np.float32)
        assert p.size == MLP_NPARAM
        self.ctx = ctx
        self.h = c_void_p()
        ctx.check(ctx.lib.diaf_model_create(ctx.h, p.ctypes.data_as(c_void_p), ctypes.byref(self.h)))

    def params(self) -> np.ndarray:
        out = np.empty(MLP_NPARAM, dtype=np.float32)
        self.ctx.check(self.ctx.lib.diaf_model_get_params(self.ctx.h, self.h,
                                                          out.ctypes.data_as(c_void_p)))
        return out

    def close(self):
        if self.h:
            self.ctx.lib.diaf_model_destroy(self.h)
            self.h = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def diaf_features(ctx: Context, A: DeviceCSC, C: DevicePattern, feat):
    ctx.check(ctx.lib.diaf_features(ctx.h, ctypes.byref(A.desc), ctypes.byref(C.desc),
                                    c_void_p(feat.data_ptr())))


def diaf_labels(ctx: Context, A: DeviceCSC, F: Factors, tau: float, labels):
    ctx.check(ctx.lib.diaf_labels(ctx.h, ctypes.byref(A.desc), F.h, tau,
                                  c_void_p(labels.data_ptr())))


def diaf_mlp_forward(ctx: Context, m: Model, feat, npairs: int, scores):
    ctx.check(ctx.lib.diaf_mlp_forward(ctx.h, m.h, c_void_p(feat.data_ptr()), npairs,
                                       c_void_p(scores.data_ptr())))


def diaf_mlp_loss_grad(ctx: Context, m: Model, feat, labels, npairs: int, grad=None) -> float:
    loss = c_double()
    ctx.check(ctx.lib.diaf_mlp_loss_grad(ctx.h, m.h, c_void_p(feat.data_ptr()),
                                         c_void_p(labels.data_ptr()), npairs,
                                         c_void_p(grad.data_ptr()) if grad is not None else None,
                                         ctypes.byref(loss)))
    return loss.value


def diaf_mlp_train_step(ctx: Context, m: Model, feat, labels, npairs: int, lr: float) -> float:
    loss = c_double()
    ctx.check(ctx.lib.diaf_mlp_train_step(ctx.h, m.h, c_void_p(feat.data_ptr()),
                                          c_void_p(labels.data_ptr()), npairs, lr,
                                          ctypes.byref(loss)))
    return loss.value
