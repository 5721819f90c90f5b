"""Host-side checks of the C ABI library (no GPU compute).

The library must load, export every function declared in include/diaf.h,
and the Python binding must declare exactly those names.
"""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "diaf.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(diaf_[a-z0-9_]+)\s*\(", src)
    return sorted(set(names))


def test_header_declares_the_api():
    names = declared_functions()
    for must in ("diaf_ctx_create", "diaf_factor", "diaf_apply", "diaf_solve",
                 "diaf_factors_view", "diaf_model_create", "diaf_mlp_train_step"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_1208_3573_amd import diaf
    lib = diaf.load_library()
    for name in declared_functions():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", diaf.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (diaf_\w+)", out))
    assert set(declared_functions()) <= exported
    # the binding marshals exactly the declared API
    assert set(diaf.EXPORTED) == set(declared_functions())


def test_binding_fails_loudly_without_library(tmp_path):
    from paper_1208_3573_amd import diaf
    saved = diaf._lib
    diaf._lib = None
    try:
        with pytest.raises(RuntimeError, match="not built"):
            diaf.load_library(str(tmp_path / "missing.so"))
    finally:
        diaf._lib = saved


def test_struct_layouts_match_header():
    """ctypes mirrors of the ABI structs have the C sizes (LP64)."""
    import ctypes
    from paper_1208_3573_amd import diaf
    assert ctypes.sizeof(diaf.diaf_csc) == 8 + 8 + 8 + 8 + 8 + 8
    assert ctypes.sizeof(diaf.diaf_pattern) == 32
    assert ctypes.sizeof(diaf.diaf_solve_info) == 4 + 4 + 8 + 8 + 8
    assert ctypes.sizeof(diaf.diaf_sparsify) == 4 * 4 + 8 + 8 + 8
    assert diaf.diaf_spec.sparsify.offset == 80 and diaf.diaf_spec.v_blocks.offset == 120
    assert diaf.diaf_spec.left.offset == 132 and ctypes.sizeof(diaf.diaf_spec) == 136
    assert diaf.MLP_NPARAM == 5313


def test_null_arguments_are_rejected_without_a_device():
    """Argument checks run before any device work and return codes only."""
    import ctypes
    from paper_1208_3573_amd import diaf
    lib = diaf.load_library()
    assert lib.diaf_ctx_create(None, 0, None) == diaf.DIAF_EINVAL
    assert lib.diaf_factor(None, None, None, 0, None) == diaf.DIAF_EINVAL
    assert lib.diaf_factors_view(None, None) == diaf.DIAF_EINVAL
    assert lib.diaf_apply(None, None, None, None) == diaf.DIAF_EINVAL
    assert lib.diaf_last_error(None) == b""
    lib.diaf_factors_destroy(None)
    lib.diaf_model_destroy(None)
    lib.diaf_ctx_destroy(None)
    h = ctypes.c_void_p()
    rc = lib.diaf_ctx_create(ctypes.byref(h), 0, None)
    if rc == diaf.DIAF_OK:  # a GPU is present: clean up
        lib.diaf_ctx_destroy(h)
    else:
        assert rc == diaf.DIAF_EDEVICE


def test_struct_layouts_match_the_c_compiler(tmp_path):
    """Sizes and field offsets of the ctypes mirrors against the C compiler's
    own layout of include/diaf.h (gcc, host code only)."""
    import ctypes
    from paper_1208_3573_amd import diaf
    structs = {"diaf_csc": diaf.diaf_csc, "diaf_pattern": diaf.diaf_pattern,
               "diaf_solve_info": diaf.diaf_solve_info, "diaf_stats": diaf.diaf_stats,
               "diaf_spec": diaf.diaf_spec, "diaf_view": diaf.diaf_view,
               "diaf_sparsify": diaf.diaf_sparsify}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "diaf.h"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append(f'printf("{name} %zu\\n", sizeof({name}));')
        for fname, _ in cls._fields_:
            lines.append(f'printf("{name}.{fname} %zu\\n", offsetof({name}, {fname}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout
    got = dict(line.rsplit(" ", 1) for line in out.strip().splitlines())
    for name, cls in structs.items():
        assert int(got[name]) == ctypes.sizeof(cls), name
        for fname, _ in cls._fields_:
            assert int(got[f"{name}.{fname}"]) == getattr(cls, fname).offset, (name, fname)
