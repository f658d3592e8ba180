"""The C-ABI library loads and exports every entry point include/gw.h declares;
host-side argument checks reject bad input before any device work (these
calls never reach the GPU, so they run without one)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gw.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gw_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    import paper_2509_23018_amd as gw
    if not os.path.exists(gw.library_path):
        pytest.fail("libgw.so is not built (python -m paper_2509_23018_amd.build)")
    return gw.lib()


def test_header_declares_the_boundary():
    names = _declared()
    for want in ("gw_mtxel", "gw_chi0", "gw_chi0_backward", "gw_last_error", "gw_release",
                 "gw_abi_version"):
        assert want in names


def test_library_exports_every_declared_symbol(lib):
    for name in _declared():
        assert hasattr(lib, name), name
    assert lib.gw_abi_version() == 1


def _grid(gw, n, vol=1000.0):
    g = gw._Grid()
    for i in range(3):
        g.n[i] = n[i]
    g.volume = vol
    return g


@pytest.mark.parametrize("n,gvec,begin,count,msg", [
    ((8, 8, 8), [[0, 0, 0], [4, 0, 0]], 0, 1, "outside"),
    ((8, 8, 8), [[0, 0, 0], [-5, 0, 0]], 0, 1, "outside"),
    ((7, 8, 8), [[3, 0, 0], [-4, 0, 0]], 0, 1, "outside"),
    ((8, 8, 8), [[1, 2, 3], [1, 2, 3]], 0, 1, "duplicate"),
    ((8, 8, 8), [[0, 0, 0]], 3, 2, "pair range"),
    ((8, 8, 8), [[0, 0, 0]], -1, 1, "pair range"),
    ((0, 8, 8), [[0, 0, 0]], 0, 1, "dimension"),
])
def test_mtxel_argument_checks(lib, n, gvec, begin, count, msg):
    import paper_2509_23018_amd as gw
    g = np.ascontiguousarray(np.array(gvec, np.int32))
    grid = _grid(gw, n)
    st = lib.gw_mtxel(ctypes.byref(grid), 16, 2, 16, 2, g.ctypes.data, g.shape[0], begin, count,
                      16, None)
    assert st == -1
    assert msg in lib.gw_last_error().decode()


def test_chi0_argument_checks(lib):
    import paper_2509_23018_amd as gw
    p = gw._Problem()
    p.grid = _grid(gw, (8, 8, 8))
    g = np.zeros((1, 3), np.int32)
    z = np.zeros(1, np.complex128)
    p.psi_v = p.psi_c = p.e_v = p.e_c = p.chi = 16
    p.nv, p.nc = 2, 2
    p.gvec, p.ng, p.z, p.nz = g.ctypes.data, 1, z.ctypes.data, 1
    o = gw._opts(pair_chunk=-1)
    assert lib.gw_chi0(ctypes.byref(p), 1, ctypes.byref(o), None) == -1
    assert "pair_chunk" in lib.gw_last_error().decode()
    o = gw._opts(precision=9)
    assert lib.gw_chi0(ctypes.byref(p), 1, ctypes.byref(o), None) == -1
    o = gw._opts()
    p.nz = 0
    assert lib.gw_chi0(ctypes.byref(p), 1, ctypes.byref(o), None) == -1
    assert "nz" in lib.gw_last_error().decode()
    p.nz = 1
    p.psi_v = None
    assert lib.gw_chi0(ctypes.byref(p), 1, ctypes.byref(o), None) == -1
    assert lib.gw_chi0(None, 1, ctypes.byref(o), None) == -1
    assert lib.gw_chi0_backward(None, None, None, None, None, None, None, None) == -1
