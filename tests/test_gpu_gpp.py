"""The GPP off-diagonal self-energy kernel (full Sigma_lm(E) on an energy
grid, the GEMM pair per band and energy with the plasmon-pole matrix formed
inside the first GEMM) against the FP64 oracle."""
import numpy as np
import pytest
import torch

import oracle
import paper_2509_23018_amd as gw
from gpu_helpers import FP64_TOL, device, rel_fro
from workloads import gen

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("nb,ns,ng,ne", [(5, 70, 150, 4), (3, 8, 64, 1), (2, 129, 65, 3)])
def test_gpp_sigma_matches_oracle(nb, ns, ng, ne):
    """Ragged tiles on both GEMMs (N_Sigma and N_G off multiples of 64),
    occupied and empty bands, complex energies."""
    inp = gen.gpp_inputs(nb, ns, ng, ne, seed=ns + ng)
    want = oracle.gpp_sigma_offdiag(inp["m"], inp["e_n"], inp["occupied"], inp["energies"],
                                     inp["omega2"], inp["wtilde"], inp["v"])
    d = {k: torch.from_numpy(np.ascontiguousarray(inp[k])).to(device())
         for k in ("m", "omega2", "wtilde", "v")}
    got = gw.gw_gpp_sigma(d["m"], inp["e_n"], inp["occupied"], inp["energies"], d["omega2"],
                          d["wtilde"], d["v"]).cpu().numpy()
    assert got.shape == (ne, ns, ns)
    assert rel_fro(got, want) < FP64_TOL, rel_fro(got, want)
    for i in range(ne):
        assert rel_fro(got[i], want[i]) < FP64_TOL


def test_gpp_sigma_no_bands_and_errors():
    inp = gen.gpp_inputs(2, 4, 16, 2, seed=3)
    d = {k: torch.from_numpy(np.ascontiguousarray(inp[k])).to(device())
         for k in ("m", "omega2", "wtilde", "v")}
    got = gw.gw_gpp_sigma(d["m"][:0], inp["e_n"][:0], inp["occupied"][:0], inp["energies"],
                          d["omega2"], d["wtilde"], d["v"])
    assert torch.all(got == 0)
    with pytest.raises((gw.GWError, ValueError)):
        gw.gw_gpp_sigma(d["m"], inp["e_n"][:1], inp["occupied"], inp["energies"], d["omega2"],
                        d["wtilde"], d["v"])
