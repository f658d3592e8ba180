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
    for want in ("gw_mtxel", "gw_chi0", "gw_chi0_backward", "gw_workspace_bytes",
                 "gw_pseudobands_workspace_bytes", "gw_last_error", "gw_release",
                 "gw_abi_version"):
        assert want in names


def test_library_exports_every_declared_symbol(lib):
    for name in _declared():
        assert hasattr(lib, name), name
    assert lib.gw_abi_version() == 2


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
    o = gw._opts(flags=gw.GW_FLAG_ACC_HERMITIAN)
    assert lib.gw_chi0(ctypes.byref(p), 1, ctypes.byref(o), None) == -1
    assert "GW_FLAG_ACCUMULATE" in lib.gw_last_error().decode()
    o = gw._opts()
    p.psi_v = None
    assert lib.gw_chi0(ctypes.byref(p), 1, ctypes.byref(o), None) == -1
    assert lib.gw_chi0(None, 1, ctypes.byref(o), None) == -1
    assert lib.gw_chi0_backward(None, None, None, None, None, None, None, None) == -1


def _pb(lib, nb=4, nr=16, keep=(), idx=(0, 1, 2), off=(0, 3), n_xi=2, theta=None,
        ws=None, ws_bytes=0):
    """gw_pseudobands with host tables and dummy device pointers (the
    argument checks run on the host before anything touches them)."""
    k = np.asarray(keep, np.int32)
    ix = np.asarray(idx, np.int32)
    of = np.asarray(off, np.int32)
    th = np.zeros(max(1, len(ix) * n_xi)) if theta is None else np.asarray(theta, np.float64)
    st = lib.gw_pseudobands(16, 16, nb, nr, k.ctypes.data if len(k) else None, len(k),
                            ix.ctypes.data, of.ctypes.data, len(of) - 1, n_xi, th.ctypes.data,
                            16, 16, ws, ws_bytes, None)
    return st, lib.gw_last_error().decode()


def test_pseudobands_argument_checks(lib):
    assert _pb(lib, off=(0, 3, 3), idx=(0, 1, 2)) == (-1, "slice 1 is empty")
    assert _pb(lib, off=(1, 3))[0] == -1
    st, msg = _pb(lib, idx=(0, 1, 4))
    assert st == -1 and "out of range" in msg
    st, msg = _pb(lib, keep=(7,))
    assert st == -1 and "out of range" in msg
    st, msg = _pb(lib, n_xi=9)
    assert st == -1 and "n_xi" in msg
    st, msg = _pb(lib, theta=[0.0, np.nan, 0.0, 0.0, 0.0, 0.0])
    assert st == -1 and "finite" in msg
    st, msg = _pb(lib, nr=1 << 31)
    assert st == -1 and "2^31" in msg
    n = 65536
    st, msg = _pb(lib, nb=n, idx=np.arange(n), off=np.arange(n + 1), n_xi=1)
    assert st == -4 and "65535" in msg
    # nothing to produce: returns before any device work
    z = np.zeros(1, np.int32)
    assert lib.gw_pseudobands(None, None, 0, 1, None, 0, None, z.ctypes.data, 0, 2, None,
                              None, None, None, 0, None) == 0


def test_pseudobands_workspace(lib):
    """The workspace size grows with the tables, and a workspace one byte too
    small, or not 256-byte aligned, is rejected on the host before any
    device work."""
    need = lib.gw_pseudobands_workspace_bytes(0, 3, 1, 2)
    assert 0 < need < 4096
    assert lib.gw_pseudobands_workspace_bytes(5, 300, 7, 4) > need
    assert lib.gw_pseudobands_workspace_bytes(-1, 3, 1, 2) == ctypes.c_size_t(-1).value
    st, msg = _pb(lib, ws=1 << 20, ws_bytes=need - 1)
    assert st == -1 and "too small" in msg
    st, msg = _pb(lib, ws=(1 << 20) + 64, ws_bytes=need)
    assert st == -1 and "aligned" in msg


def test_workspace_query_argument_checks(lib):
    """gw_workspace_bytes runs the same host checks as gw_chi0 and returns
    SIZE_MAX with a message when they fail."""
    import paper_2509_23018_amd as gw
    bad = ctypes.c_size_t(-1).value
    p = gw._Problem()
    p.grid = _grid(gw, (8, 8, 8))
    g = np.array([[0, 0, 0], [0, 0, 0]], np.int32)
    z = np.zeros(1, np.complex128)
    p.psi_v = p.psi_c = p.e_v = p.e_c = p.chi = 16
    p.nv, p.nc = 2, 2
    p.gvec, p.ng, p.z, p.nz = g.ctypes.data, 2, z.ctypes.data, 1
    o = gw._opts()
    assert lib.gw_workspace_bytes(ctypes.byref(p), 1, ctypes.byref(o), 0) == bad
    assert "duplicate" in lib.gw_last_error().decode()
    assert lib.gw_workspace_bytes(ctypes.byref(p), 1, ctypes.byref(o), 1) == bad
    assert lib.gw_workspace_bytes(None, 1, ctypes.byref(o), 0) == bad
    assert lib.gw_workspace_bytes(ctypes.byref(p), 0, ctypes.byref(o), 1) == bad
    o = gw._opts(precision=7)
    p.ng = 1
    assert lib.gw_workspace_bytes(ctypes.byref(p), 1, ctypes.byref(o), 0) == bad
    assert "precision" in lib.gw_last_error().decode()
    # a misaligned workspace is an argument error of gw_chi0 itself
    o = gw._opts()
    o.workspace, o.workspace_bytes = (1 << 20) + 8, 1 << 20
    assert lib.gw_chi0(ctypes.byref(p), 1, ctypes.byref(o), None) == -1
    assert "aligned" in lib.gw_last_error().decode()


def test_pseudoband_recipe():
    """The recipe protects the lowest energies and cuts the rest, in energy
    order, into consecutive slices of the given sizes; the phases are in
    [0, 1) with one row per pseudoband."""
    from workloads import gen
    rng = np.random.default_rng(2)
    e = rng.random(40)
    keep, slices, theta = gen.pseudoband_recipe(e, 6, [4, 10, 20], 3, seed=9)
    order = np.argsort(e, kind="stable")
    assert np.array_equal(keep, order[:6])
    assert np.array_equal(np.concatenate(slices), order[6:])
    assert [len(s) for s in slices] == [4, 10, 20]
    for a, b in zip(slices[:-1], slices[1:]):
        assert e[a].max() <= e[b].min()
    assert [t.shape for t in theta] == [(3, 4), (3, 10), (3, 20)]
    assert all(((t >= 0) & (t < 1)).all() for t in theta)
    _, _, again = gen.pseudoband_recipe(e, 6, [4, 10, 20], 3, seed=9)
    assert all(np.array_equal(a, b) for a, b in zip(theta, again))
    with pytest.raises(ValueError):
        gen.pseudoband_recipe(e, 6, [4, 10], 3, seed=9)
