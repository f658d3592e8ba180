"""GPU parity of gw_mtxel against the FP64 oracle (element by element)."""
import itertools
import math

import numpy as np
import pytest
import torch

import oracle
import paper_2509_23018_amd as gw
from gpu_helpers import FP64_TOL, device, rel_fro
from workloads import gen

pytestmark = pytest.mark.gpu
VOL = 1000.0


def _all_g(n):
    axes = [range(-(k // 2), k - k // 2) for k in n]
    return np.array(list(itertools.product(*axes)), dtype=np.int32)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device())


@pytest.mark.parametrize("n,nv,nc,r2", [
    ((16, 16, 16), 4, 28, 10),      # workload 0 shape
    ((12, 10, 9), 3, 5, 8),         # non-cubic, odd axis
    ((24, 24, 24), 2, 7, 40),       # |g| <= 6: 13 values (7 classes) per axis, one block
    ((36, 20, 44), 2, 3, 90),       # 19 k3 values, 10 classes: two blocks, N2 not a multiple of 16
    ((8, 8, 8), 1, 3, 20),          # sphere clipped by the grid: keeps g = -4, drops g = +4
])
def test_mtxel_matches_oracle(n, nv, nc, r2):
    p = gen.make_problem(n, nv, nc, r2=r2, seed=sum(n))
    g = gen.gsphere(r2)
    nn = np.array(n)
    lo, hi = -(nn // 2), (nn + 1) // 2 - 1
    g = g[np.all((g >= lo) & (g <= hi), axis=1)]
    m = gw.gw_mtxel(_dev(p.psi_v), _dev(p.psi_c), g, n, p.volume).cpu().numpy()
    ref = oracle.mtxel(p.psi_v, p.psi_c, g, n, p.volume)
    assert m.shape == ref.shape
    assert rel_fro(m, ref) < FP64_TOL


def test_mtxel_full_grid_and_pair_range():
    n = (6, 8, 5)
    p = gen.make_problem(n, 3, 4, gvec=_all_g(n), seed=3)
    m = gw.gw_mtxel(_dev(p.psi_v), _dev(p.psi_c), p.gvec, n, p.volume, pair_begin=5,
                    pair_count=6).cpu().numpy()
    ref = oracle.mtxel(p.psi_v, p.psi_c, p.gvec, n, p.volume, pairs=range(5, 11))
    assert rel_fro(m, ref) < FP64_TOL


def test_mtxel_pair_range_rectangles():
    """A pair range that starts and ends inside a row and spans whole rows of
    more than 1,024 conduction bands: it is cut into a partial row, blocks of 4
    valence bands split into column ranges, a single row and a partial row,
    written at their places in the linear pair order."""
    n = (8, 6, 5)
    nv, nc = 7, 1100
    p = gen.make_problem(n, nv, nc, r2=3, seed=11, orthonormalize=False)
    b, cnt = 1000, 6 * nc + 50
    m = gw.gw_mtxel(_dev(p.psi_v), _dev(p.psi_c), p.gvec, n, p.volume, pair_begin=b,
                    pair_count=cnt).cpu().numpy()
    ref = oracle.mtxel(p.psi_v, p.psi_c, p.gvec, n, p.volume, pairs=range(b, b + cnt))
    assert rel_fro(m, ref) < FP64_TOL


def test_mtxel_plane_waves_exact():
    n = (16, 12, 10)
    kv = [(0, 0, 0), (3, -2, 4), (-8, 5, -5)]
    kc = [(1, 0, 0), (3, -2, 3), (7, 5, 4), (0, 1, -1)]
    j = np.meshgrid(*[np.arange(k) for k in n], indexing="ij")

    def pw(ks):
        return np.array([np.exp(2j * np.pi * sum(k[a] * j[a] / n[a] for a in range(3))).reshape(-1)
                         / math.sqrt(VOL) for k in ks])

    g = _all_g(n)
    m = gw.gw_mtxel(_dev(pw(kv)), _dev(pw(kc)), g, n, VOL).cpu().numpy()
    nn = np.array(n)
    for v, c in itertools.product(range(len(kv)), range(len(kc))):
        want = np.all((g % nn) == (np.array(kv[v]) - np.array(kc[c])) % nn, axis=1).astype(float)
        assert np.abs(m[v * len(kc) + c] - want).max() < 1e-12


def test_mtxel_completeness_with_aliased_windows():
    """psi_c = all N_r states, psi_v a window of the same array: sum_n |M_vn|^2 = 1."""
    n = (4, 4, 4)
    nr = 64
    rng = np.random.default_rng(2)
    psi = gen.orthonormal_bands(rng, nr, n, VOL)
    g = _all_g(n)[::3]
    dpsi = _dev(psi)
    m = gw.gw_mtxel(dpsi[:5], dpsi, g, n, VOL).cpu().numpy().reshape(5, nr, -1)
    assert np.abs(np.sum(np.abs(m) ** 2, axis=1) - 1.0).max() < 1e-12


def test_mtxel_rejects_bad_arguments():
    n = (8, 8, 8)
    psi = _dev(np.zeros((2, 512), np.complex128))
    out = torch.full((2, 2), 7.0 + 0j, dtype=torch.complex128, device=device())
    with pytest.raises(gw.GWError, match="outside"):
        gw.gw_mtxel(psi, psi, np.array([[0, 0, 0], [4, 0, 0]]), n, VOL, 0, 2, out=out)
    with pytest.raises(gw.GWError, match="duplicate"):
        gw.gw_mtxel(psi, psi, np.array([[1, 0, 0], [1, 0, 0]]), n, VOL, 0, 2, out=out)
    with pytest.raises(gw.GWError, match="pair range"):
        gw.gw_mtxel(psi, psi, np.array([[0, 0, 0], [1, 0, 0]]), n, VOL, 3, 2, out=out)
    torch.cuda.synchronize()
    assert torch.all(out == 7.0)        # untouched on error


def _box_g(r1, r2, r3):
    """Miller indices of the box r1 x r2 x r3 (inclusive ranges)."""
    axes = [np.arange(lo, hi + 1) for lo, hi in (r1, r2, r3)]
    return np.array(list(itertools.product(*axes)), dtype=np.int32)


@pytest.mark.parametrize("n,g", [
    ((6, 10, 16), _box_g((-2, 2), (-4, 3), (-8, 7))),     # N3 = 16: the whole k3 window
    ((5, 9, 32), _box_g((-2, 2), (-4, 4), (-7, 7))),      # N3 = 32
    ((7, 12, 48), _box_g((-3, 3), (-6, 5), (-8, 5))),     # N3 = 48, window not centred: unpaired k3
    ((4, 24, 64), _box_g((-1, 1), (-10, 10), (-6, 6))),   # N3 = 64, 21 k2 values: two y blocks
    # more than 24 classes on both the y and z axes: four class blocks each
    # (and 26 x 19), the stage-y accumulators beyond the registers of a wave
    ((3, 52, 52), _box_g((-1, 1), (-25, 25), (-25, 25))),
    ((3, 52, 40), _box_g((-1, 1), (-25, 25), (-18, 18))),
])
def test_mtxel_box_g_lists(n, g):
    """Box-shaped G lists with holes on grids with N3 from 16 to 64, the k3
    values filling the window [-8, 7] or part of it off centre, 21 k2 values
    (two y-stage blocks), and 26 classes on y with 26 or 19 on z (the largest
    stage-y blocks): against the oracle, with ragged pair tiles (3 valence x
    37 conduction bands)."""
    keep = np.ones(len(g), bool)
    keep[::7] = False                    # holes in the disc
    g = np.ascontiguousarray(g[keep])
    p = gen.make_problem(n, 3, 37, gvec=g, seed=sum(n))
    m = gw.gw_mtxel(_dev(p.psi_v), _dev(p.psi_c), g, n, p.volume).cpu().numpy()
    ref = oracle.mtxel(p.psi_v, p.psi_c, g, n, p.volume)
    assert rel_fro(m, ref) < FP64_TOL
