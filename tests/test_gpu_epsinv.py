"""The inverse dielectric matrix of Eq. (3), eps^-1 = [I - v chi]^-1, on the
device (block Gauss-Jordan on FP64 MFMA GEMMs) against the FP64 oracle."""
import numpy as np
import pytest
import torch

import oracle
import paper_2509_23018_amd as gw
from gpu_helpers import FP64_TOL, device, rel_fro, to_dev
from workloads import gen

pytestmark = pytest.mark.gpu


def _chi_problem(seed, n=(16, 16, 16), nv=3, nc=30, r2=20, z=(0.0, 0.5j, 2.0j, 0.2 + 0.05j)):
    p = gen.make_problem(n, nv, nc, r2=r2, z=z, seed=seed, pair_chunk=64)
    chi = oracle.chi0(p.psi_v, p.psi_c, p.e_v, p.e_c, p.gvec, p.z, p.n, p.volume,
                      spin=p.spin, pair_chunk=p.pair_chunk)
    return p, chi


@pytest.mark.parametrize("seed,r2", [(51, 20), (52, 30), (53, 6)])
def test_epsinv_matches_oracle(seed, r2):
    """Several 64-wide blocks and a ragged one (N_G = 389, 739; 57 below one
    block), zero, imaginary and real frequencies, q = 0 (the head excluded)."""
    p, chi = _chi_problem(seed, r2=r2)
    v = oracle.coulomb(p.gvec, cell_l=gen.CELL_L)
    want = oracle.epsilon_inverse(chi, v)
    got = gw.gw_epsinv(torch.from_numpy(chi).to(device()),
                       torch.from_numpy(v).to(device())).cpu().numpy()
    for w in range(len(p.z)):
        assert rel_fro(got[w], want[w]) < FP64_TOL, (w, rel_fro(got[w], want[w]))
    assert np.abs(got[:, 0, :] - np.eye(p.ng)[0]).max() < 1e-12


def test_epsinv_shifted_q_and_device_chi():
    """q != 0 (every v_G finite) with chi from the device build, and
    eps eps^-1 = I checked on the device."""
    p, chi = _chi_problem(54, r2=15, z=(0.0, 0.8j))
    q = (0.125, -0.25, 0.375)
    v = oracle.coulomb(p.gvec, q=q, cell_l=gen.CELL_L)
    chi_d = gw.gw_chi0(to_dev(p), pair_chunk=p.pair_chunk)
    vd = torch.from_numpy(v).to(device())
    got = gw.gw_epsinv(chi_d, vd)
    want = oracle.epsilon_inverse(chi, v)
    assert rel_fro(got.cpu().numpy(), want) < FP64_TOL
    eps = torch.eye(p.ng, dtype=torch.complex128, device=device())[None] - vd[None, :, None] * chi_d
    prod = gw.gw_zgemm("N", "N", eps.contiguous(), got)
    eye = np.broadcast_to(np.eye(p.ng), prod.shape)
    assert np.abs(prod.cpu().numpy() - eye).max() < 1e-12


def test_epsinv_identity_and_errors():
    ng = 70
    chi = torch.zeros((2, ng, ng), dtype=torch.complex128, device=device())
    v = torch.ones(ng, dtype=torch.float64, device=device())
    got = gw.gw_epsinv(chi, v).cpu().numpy()
    assert np.abs(got - np.eye(ng)[None]).max() == 0.0
    with pytest.raises((gw.GWError, ValueError)):
        gw.gw_epsinv(chi, v[:5])
    with pytest.raises((gw.GWError, ValueError)):
        gw.gw_epsinv(chi[:, :, :5], v)
