"""The C-ABI library loads on a host without a GPU, exports every function
include/nexels.h declares, and rejects bad arguments before touching HIP."""
from __future__ import annotations

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nexels.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(nx_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2512_13796_amd import _lib
    return _lib.load()


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("nx_create", "nx_destroy", "nx_workspace_size", "nx_render_forward", "nx_render_backward",
                 "nx_last_error"):
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    for name in _declared():
        assert hasattr(lib, name), name


def test_binding_covers_every_symbol():
    from paper_2512_13796_amd import _lib
    assert sorted(_lib.SIGNATURES) == _declared()


def test_invalid_arguments_are_rejected_on_the_host(lib):
    from paper_2512_13796_amd import _lib as L
    h = ctypes.c_void_p()
    assert lib.nx_create(ctypes.byref(h), 3, 16, L.NX_F32, L.NX_F32) == L.NX_ERR_UNSUPPORTED
    assert b"K must be" in lib.nx_last_error()
    assert lib.nx_create(ctypes.byref(h), -1, 16, L.NX_F32, L.NX_F32) == L.NX_ERR_INVALID
    assert lib.nx_create(ctypes.byref(h), 4, 8, L.NX_F32, L.NX_F32) == L.NX_ERR_UNSUPPORTED
    assert lib.nx_create(ctypes.byref(h), 4, 16, L.NX_F32, L.NX_F16) == L.NX_ERR_UNSUPPORTED
    assert lib.nx_create(None, 4, 16, L.NX_F32, L.NX_F32) == L.NX_ERR_INVALID
    size = ctypes.c_size_t()
    cam = L.NxCamera()
    assert lib.nx_workspace_size(None, 10, ctypes.byref(cam), 1, 0, ctypes.byref(size)) == L.NX_ERR_INVALID
    out = L.NxFwdOut()
    assert lib.nx_render_forward(None, None, None, 1, None, None, ctypes.byref(out), None, 0, None,
                                 None) == L.NX_ERR_INVALID
    assert lib.nx_render_backward(None, None, None, 1, None, None, None, None, 0, None, None, None, None,
                                  None) == L.NX_ERR_INVALID
    batch = ctypes.c_int32()
    assert lib.nx_autotune_raster(None, None, None, 1, None, None, 0, 3, ctypes.byref(batch),
                                  None) == L.NX_ERR_INVALID
    assert lib.nx_fps(None, None, 10, 5, None, None, None, 0, None) != L.NX_OK
    assert lib.nx_aux_losses(None, 10, None, None, None, 0, None, None, None, None, None, None, None, None,
                             None) == L.NX_ERR_INVALID
    assert lib.nx_debug_limits(None, 0, 0) == L.NX_ERR_INVALID
    assert lib.nx_set_sh_degree(None, 3) == L.NX_ERR_INVALID
    assert lib.nx_destroy(None) == L.NX_OK
    assert lib.nx_version() >= 100


def test_struct_sizes_match_the_header():
    from paper_2512_13796_amd import _lib as L
    assert ctypes.sizeof(L.NxCamera) == 12 * 8 + 5 * 8 + 2 * 4
    assert ctypes.sizeof(L.NxHashGrid) == 32
    assert ctypes.sizeof(L.NxMLP) == 48
    assert ctypes.sizeof(L.NxFwdOut) == 12 * 8
    assert ctypes.sizeof(L.NxSurfels) == 7 * 8
    assert ctypes.sizeof(L.NxGrads) == 12 * 8


def test_one_hip_runtime_whatever_the_import_order():
    """Importing the package before torch must not map a second HIP runtime next to torch's own copy (the
    second one to open the device finds none)."""
    import subprocess
    import sys
    code = ("import paper_2512_13796_amd, torch\n"
            "print(sorted({l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l}))\n")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    out = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr[-2000:]
    import ast
    mapped = ast.literal_eval(out.stdout.strip().splitlines()[-1])
    assert len(mapped) == 1, mapped
