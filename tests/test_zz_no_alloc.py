"""gw_chi0_fixed, the entry point that allocates nothing (its scratch is a
fixed device array), against gw_chi0 and the FP64 oracle."""
import numpy as np
import pytest
import torch

import oracle
import paper_2509_23018_amd as gw
from gpu_helpers import FP64_TOL, device, rel_fro, to_dev
from workloads import gen

pytestmark = pytest.mark.gpu


def _problem(n, nv, nc, r2, seed, chunk=4096):
    return gen.make_problem(n, nv, nc, r2=r2, z=(0.0, 0.5j, 0.3 + 0.01j), seed=seed,
                            pair_chunk=chunk)


@pytest.mark.parametrize("prec,ns,tol", [("fp64", 0, FP64_TOL), ("split_bf16", 5, 1e-10)])
def test_fixed_scratch_two_calls_second_smaller(prec, ns, tol):
    """Two calls in a row, the second on a smaller problem (fewer bands and
    G-vectors, another grid), each against gw_chi0 on the same inputs (the
    ordinary entry point also builds the plan the fixed one needs) and against
    the oracle."""
    kw = dict(precision=prec, n_slices=ns)
    for n, nv, nc, r2, seed, chunk in [((20, 18, 24), 5, 60, 15, 1, 100),
                                       ((12, 12, 12), 3, 20, 9, 2, 4096)]:
        p = _problem(n, nv, nc, r2, seed, chunk)
        ref = gw.gw_chi0(to_dev(p), pair_chunk=chunk, **kw).cpu().numpy()
        dp = to_dev(p)
        dp.chi = torch.full((len(p.z), p.ng, p.ng), 3.0 + 3.0j, dtype=torch.complex128,
                            device=device())
        got = gw.gw_chi0_fixed(dp, pair_chunk=chunk, **kw)
        torch.cuda.synchronize()
        got = got.cpu().numpy()
        assert rel_fro(got, ref) < tol, (n, rel_fro(got, ref))
        want = oracle.chi0(p.psi_v, p.psi_c, p.e_v, p.e_c, p.gvec, p.z, p.n, p.volume,
                           spin=p.spin, pair_chunk=chunk)
        assert rel_fro(got, want) < tol


def test_fixed_scratch_smaller_chunks_than_requested():
    """A problem whose 4,096-pair chunks do not fit the fixed scratch runs in
    smaller chunks: same chi as gw_chi0 to rounding."""
    p = gen.make_problem((24, 24, 24), 8, 600, r2=27, z=(0.0, 0.7j), seed=3, pair_chunk=4096)
    dp = to_dev(p)
    kw = dict(pair_chunk=4096)
    assert gw.workspace_bytes(dp, **kw) > gw.lib().gw_chi0_fixed_scratch_bytes()
    ref = gw.gw_chi0(dp, **kw).clone()
    got = gw.gw_chi0_fixed(to_dev(p), **kw)
    assert rel_fro(got.cpu().numpy(), ref.cpu().numpy()) < FP64_TOL


def test_fixed_scratch_refuses_what_would_allocate():
    """A grid and G list without a plan, a caller workspace, graph capture:
    GW_EINVAL before anything runs, the output untouched."""
    p = _problem((14, 10, 12), 2, 7, 6, 4)
    dp = to_dev(p)
    dp.chi = torch.full((len(p.z), p.ng, p.ng), 2.0 + 0j, dtype=torch.complex128, device=device())
    with pytest.raises(gw.GWError) as ei:
        gw.gw_chi0_fixed(dp)
    assert ei.value.status == -1 and "allocates nothing" in str(ei.value)
    with pytest.raises(gw.GWError):
        gw.gw_chi0_fixed(dp, flags=gw.GW_FLAG_GRAPH)
    torch.cuda.synchronize()
    assert torch.all(dp.chi == 2.0)
