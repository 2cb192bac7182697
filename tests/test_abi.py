"""The C-ABI library loads and exports every entry point include/gcb.h
declares; host-side argument checks work without a GPU."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gcb.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gcb_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for want in ("gcb_load_fields", "gcb_push", "gcb_push_backward", "gcb_create",
                 "gcb_destroy", "gcb_last_error"):
        assert want in names


def test_library_exports_every_declared_symbol():
    from paper_2007_14401_amd import gcb
    lib = C.CDLL(gcb.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(gcb.EXPORTED) == set(declared_functions())


def test_null_arguments_rejected_without_device():
    from paper_2007_14401_amd import gcb
    lib = gcb.lib()
    assert lib.gcb_create(None, 0) == gcb.GCB_EINVAL
    assert "NULL" in gcb.gcb_last_error(None)
    assert lib.gcb_push(None, None, None, 1, None, None, None) == gcb.GCB_EINVAL
    assert lib.gcb_load_fields(None, None, None, None, 0, None) == gcb.GCB_EINVAL
    assert lib.gcb_push_backward(None, None, None, 1, None, None, None, None, None) in (
        gcb.GCB_EINVAL, gcb.GCB_EUNSUPPORTED)
    assert lib.gcb_kinetic_energy(None, None, None, None, None, None) == gcb.GCB_EINVAL
    assert lib.gcb_set_timing(None, 1) == gcb.GCB_EINVAL
    assert lib.gcb_load_fields_gr(None, None, None, None, 0, None) == gcb.GCB_EINVAL
    assert lib.gcb_push_gr(None, None, None, 1, None, None, None) == gcb.GCB_EINVAL
    assert lib.gcb_load_fields_3d(None, None, None, None, 0, None) == gcb.GCB_EINVAL
    assert lib.gcb_push_3d(None, None, None, 1, None, None, None) == gcb.GCB_EINVAL
    assert lib.gcb_push_backward_3d(None, None, None, 1, None, None, None, None,
                                    None) == gcb.GCB_EINVAL
    lib.gcb_destroy(None)


def test_create_without_gpu_fails_cleanly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_2007_14401_amd import gcb
    with pytest.raises(gcb.GcbError) as e:
        gcb.gcb_create(0)
    assert e.value.code in (gcb.GCB_EHIP, gcb.GCB_EINVAL)


def test_params_struct_layout_matches_header():
    """ctypes mirrors of the C structs have the sizes the header implies."""
    from paper_2007_14401_amd import gcb
    assert C.sizeof(gcb.gcb_params) == 6 * 8 + 10 * 4 + 8 + 4 + 4   # arith, keep_order
    assert C.sizeof(gcb.gcb_particles) == 8 + 10 * 8
    assert C.sizeof(gcb.gcb_grid_desc) == 4 + 4 + 8 + 8 + 96 + 8
    assert C.sizeof(gcb.gcb_stats) == 5 * 8 + 8 * 8
    assert C.sizeof(gcb.gcb_gr_desc) == 4 + 4 + 3 * 8 + 8
    assert C.sizeof(gcb.gcb_gr_particles) == 8 + 9 * 8
    assert C.sizeof(gcb.gcb_grid3_desc) == 3 * 4 + 4 + 3 * 8 + 18 * 8
    assert C.sizeof(gcb.gcb_particles3) == 8 + 12 * 8


_STRUCTS = ("gcb_grid_desc", "gcb_params", "gcb_particles", "gcb_stats", "gcb_gr_desc",
            "gcb_gr_particles", "gcb_grid3_desc", "gcb_particles3")


def test_ctypes_mirrors_match_the_c_compiler(tmp_path):
    """Every field of every public struct sits at the offset, and every
    struct has the size, that a C compiler gives the header."""
    import shutil
    import subprocess
    from paper_2007_14401_amd import gcb
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "gcb.h"', "int main(void) {"]
    for name in _STRUCTS:
        st = getattr(gcb, name)
        lines.append(f'printf("{name} size %zu\\n", sizeof({name}));')
        for f in st._fields_:
            lines.append(f'printf("{name} {f[0]} %zu\\n", offsetof({name}, {f[0]}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-I", inc, str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out.splitlines()}
    for name in _STRUCTS:
        st = getattr(gcb, name)
        assert got[(name, "size")] == C.sizeof(st), name
        for f in st._fields_:
            assert got[(name, f[0])] == getattr(st, f[0]).offset, (name, f[0])


def test_sincos_rejects_bad_arguments_without_device():
    from paper_2007_14401_amd import gcb
    lib = gcb.lib()
    assert lib.gcb_sincos(None, None, None, None, 4, None) == gcb.GCB_EINVAL
