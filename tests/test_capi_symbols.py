"""The C-ABI library builds, loads without a GPU and exports every symbol that
include/gs.h declares (no compute calls here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "gs.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?(?:gs_status|size_t|char\s*\*|void)\s*\*?\s*(gs_\w+)\s*\(",
                       src, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    from paper_2509_12138_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2509_12138_amd import build
        build.build()
    return _lib.load()


def test_header_declares_the_step():
    names = declared_functions()
    for fn in ("gs_project", "gs_bin_sort", "gs_raster_fwd", "gs_raster_bwd", "gs_project_bwd",
               "gs_loss", "gs_adam", "gs_check_status", "gs_last_error"):
        assert fn in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, f"not exported: {missing}"


def test_binding_covers_the_header():
    from paper_2509_12138_amd import _lib
    missing = [n for n in declared_functions() if n not in _lib.SIGNATURES]
    assert not missing, f"binding lacks: {missing}"


def test_host_only_calls(lib):
    from paper_2509_12138_amd import _lib
    assert lib.gs_version().startswith(b"gsmi")
    t = _lib.gs_tiling(1920, 1080, 16, 16)
    assert lib.gs_bin_sort_workspace_bytes(1000, 5000, ctypes.byref(t), 1) > 5000 * 12
    # two FP32 block sums per (image, channel, 32x32 tile)
    assert lib.gs_loss_workspace_bytes(2, 64, 64) >= 2 * 3 * 2 * 4 * 4
    # argument validation fails before anything is enqueued (no GPU needed)
    st = lib.gs_zero(None, 6, None)
    assert st == _lib.GS_ERR_ARG and b"multiple of 4" in lib.gs_last_error()
    v = _lib.gs_views(0, 0, None, None, None)
    p = _lib.gs_projected(None, None, None, 0)
    st = lib.gs_raster_fwd(ctypes.byref(p), ctypes.byref(v), ctypes.byref(t), None, None,
                           _lib.F3(0, 0, 0), None, None, None, None, None)
    assert st == _lib.GS_ERR_ARG and b"n_slots" in lib.gs_last_error()
    st = lib.gs_adam(None, 1, 0.9, 0.999, 1e-15, 0, 1, None)
    assert st == _lib.GS_ERR_ARG


def test_ctypes_structs_match_the_header_layout(tmp_path):
    """Every struct the binding mirrors has the header's size and field
    offsets (compiled with the host C compiler)."""
    import shutil
    import subprocess
    from paper_2509_12138_amd import _lib
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    structs = [n for n in dir(_lib) if n.startswith("gs_") and isinstance(getattr(_lib, n), type)
               and issubclass(getattr(_lib, n), ctypes.Structure)]
    assert "gs_gaussians" in structs and "gs_gaussian_state" in structs
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "gs.h"', 'int main(void) {']
    for s in structs:
        lines.append(f'  printf("{s} size %zu\\n", sizeof({s}));')
        for f, _ in getattr(_lib, s)._fields_:
            lines.append(f'  printf("{s} {f} %zu\\n", offsetof({s}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    for line in filter(None, out):
        s, f, v = line.split()
        cls = getattr(_lib, s)
        want = ctypes.sizeof(cls) if f == "size" else getattr(cls, f).offset
        assert int(v) == want, (s, f, int(v), want)
