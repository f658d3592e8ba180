"""GPU parity of gw_chi0_backward against the oracle adjoint and finite differences."""
import numpy as np
import pytest
import torch

import oracle
import paper_2509_23018_amd as gw
from gpu_helpers import FP64_TOL, device, rel_fro, to_dev
from workloads import gen

pytestmark = pytest.mark.gpu


def _herm(rng, nz, ng):
    x = rng.standard_normal((nz, ng, ng)) + 1j * rng.standard_normal((nz, ng, ng))
    return np.ascontiguousarray(0.5 * (x + np.conj(np.transpose(x, (0, 2, 1)))))


@pytest.mark.parametrize("zs,chunk", [((0.0,), 17), ((0.4j, 0.3 + 0.01j), 1000)])
def test_backward_matches_oracle_adjoint(zs, chunk):
    p = gen.make_problem((12, 10, 14), 4, 11, r2=9, z=zs, seed=21, pair_chunk=chunk)
    rng = np.random.default_rng(5)
    w = _herm(rng, len(p.z), p.ng)
    dp = to_dev(p)
    got = gw.gw_chi0_backward(dp, torch.from_numpy(w).to(device()), pair_chunk=chunk)
    ref = oracle.chi0_backward(p.psi_v, p.psi_c, p.e_v, p.e_c, p.gvec, p.z, p.n, p.volume, w,
                               spin=p.spin, pair_chunk=chunk)
    for g, r in zip(got, ref):
        assert rel_fro(g.cpu().numpy(), r) < FP64_TOL


def test_autograd_function_and_finite_differences():
    """L = Re tr(A chi0) through torch.autograd, against central differences."""
    p = gen.make_problem((10, 10, 10), 3, 6, r2=6, z=(0.0,), seed=8, pair_chunk=5)
    rng = np.random.default_rng(9)
    a = torch.from_numpy(_herm(rng, 1, p.ng)[0]).to(device())
    dp = to_dev(p)
    psi_v = dp.psi_v.clone().requires_grad_(True)
    psi_c = dp.psi_c.clone().requires_grad_(True)
    e_v = dp.e_v.clone().requires_grad_(True)
    e_c = dp.e_c.clone().requires_grad_(True)

    def loss(pv, pc, ev, ec):
        chi = gw.chi0(pv, pc, ev, ec, p.gvec, p.z, p.n, p.volume, pair_chunk=5)
        return torch.real(torch.trace(a @ chi[0]))

    L = loss(psi_v, psi_c, e_v, e_c)
    L.backward()
    h = 1e-6
    for which in range(4):
        base = [dp.psi_v, dp.psi_c, dp.e_v, dp.e_c]
        grad = [psi_v.grad, psi_c.grad, e_v.grad, e_c.grad][which]
        x = base[which]
        d = torch.randn_like(x)
        d = d * (x.norm() / d.norm())
        plus = list(base)
        minus = list(base)
        plus[which] = x + h * d
        minus[which] = x - h * d
        with torch.no_grad():
            fd = (loss(*plus) - loss(*minus)).item() / (2 * h)
        pred = torch.real(torch.sum(torch.conj(grad) * d)).item()
        assert abs(fd - pred) < 1e-6 * max(1.0, abs(fd)), (which, fd, pred)
