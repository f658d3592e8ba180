"""Stochastic pseudobands on the device against the oracle: the mixtures
element by element, and chi0 built from them."""
import numpy as np
import pytest
import torch

import oracle
import paper_2509_23018_amd as gw
from gpu_helpers import FP64_TOL, device, rel_fro, run_chi0
from workloads import gen

pytestmark = pytest.mark.gpu


def _bands(nb, n=(9, 8, 7), seed=5):
    """nb orthonormal bands on a ragged grid (504 points: not a multiple of
    the 64 points of a mixing workgroup or the 256 of a copy workgroup) with
    uniform energies."""
    p = gen.make_problem(n, 1, nb, r2=2, z=(0.0,), seed=seed)
    return p.psi_c, p.e_c


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(device())


@pytest.mark.parametrize("n_xi", [1, 3, 8])
def test_pseudobands_match_oracle(n_xi):
    """Protected bands, slices of 1 to 300 bands (fewer than the four waves
    that split a slice's bands, a count they do not divide, and long ones),
    bands out of order within a slice, slices not in size order."""
    psi, e = _bands(420)
    rng = np.random.default_rng(n_xi)
    perm = rng.permutation(420)
    keep = perm[:5]
    slices = [perm[5:6], perm[113:413], perm[6:13], perm[13:113]]
    theta = [rng.random((n_xi, len(s))) for s in slices]
    got, ge = gw.gw_pseudobands(_dev(psi), _dev(e), keep, slices, n_xi, theta)
    ref, re = oracle.pseudobands(psi, e, keep, slices, n_xi, theta)
    g = got.cpu().numpy()
    assert g.shape == ref.shape
    assert np.abs(g - ref).max() <= 1e-13 * np.abs(ref).max()
    assert np.array_equal(g[:5], psi[keep])
    assert np.allclose(ge.cpu().numpy(), re, rtol=1e-15, atol=0)


def test_chi0_from_pseudobands():
    """chi0 with the conduction bands compressed on the device equals the
    oracle's chi0 on the oracle's pseudobands (same phases)."""
    p = gen.make_problem((12, 12, 10), 3, 60, r2=8, z=(0.0, 0.4 + 0.01j), seed=19,
                         pair_chunk=40)
    order = np.argsort(p.e_c)
    keep, rest = order[:8], order[8:]
    slices = [rest[:12], rest[12:28], rest[28:]]
    rng = np.random.default_rng(3)
    theta = [rng.random((2, len(s))) for s in slices]
    pc, ec = gw.gw_pseudobands(_dev(p.psi_c), _dev(p.e_c), keep, slices, 2, theta)
    q = gen.Problem(**{**p.__dict__})
    q.psi_c, q.e_c = pc.cpu().numpy(), ec.cpu().numpy()
    got = run_chi0(q)
    opc, oec = oracle.pseudobands(p.psi_c, p.e_c, keep, slices, 2, theta)
    ref = oracle.chi0(p.psi_v, opc, p.e_v, oec, p.gvec, p.z, p.n, p.volume,
                      pair_chunk=p.pair_chunk)
    assert rel_fro(got, ref) < FP64_TOL


def test_pseudobands_workload1_full_size():
    """The 48^3 workload's 960 conduction bands at full size, compressed as
    the bench does (64 protected, slices of 16 to 400 bands, 4 pseudobands
    each): every element against the oracle."""
    p = gen.make_config(1)
    keep, slices, theta = gen.pseudoband_recipe(p.e_c, 64, [16, 32, 64, 128, 256, 400], 4,
                                                seed=1005)
    got, ge = gw.gw_pseudobands(_dev(p.psi_c), _dev(p.e_c), keep, slices, 4, theta)
    ref, re = oracle.pseudobands(p.psi_c, p.e_c, keep, slices, 4, theta)
    g = got.cpu().numpy()
    assert g.shape == ref.shape == (88, int(np.prod(p.n)))
    assert np.abs(g - ref).max() <= 1e-13 * np.abs(ref).max()
    assert np.allclose(ge.cpu().numpy(), re, rtol=1e-15, atol=0)


def test_pseudobands_rejects_bad_arguments():
    psi, e = _bands(10)
    dp, de = _dev(psi), _dev(e)
    th = [np.zeros((2, 3))]
    with pytest.raises(gw.GWError, match="empty"):
        gw.gw_pseudobands(dp, de, [], [np.arange(3), np.zeros(0, int)], 2, th + [np.zeros((2, 0))])
    with pytest.raises(gw.GWError, match="out of range"):
        gw.gw_pseudobands(dp, de, [10], [np.arange(3)], 2, th)
    with pytest.raises(gw.GWError, match="n_xi"):
        gw.gw_pseudobands(dp, de, [], [np.arange(3)], 9, [np.zeros((9, 3))])
    with pytest.raises(gw.GWError, match="finite"):
        gw.gw_pseudobands(dp, de, [], [np.arange(3)], 2, [np.full((2, 3), np.nan)])
    out, oe = gw.gw_pseudobands(dp, de, [], [], 2, [])
    assert out.shape[0] == 0 and oe.shape[0] == 0
