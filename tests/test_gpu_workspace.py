"""Calls that run in a caller-owned workspace (no library scratch), the
too-small-workspace error, the bounded graph cache and plan lifetimes, each
against the FP64 oracle."""
import os

import numpy as np
import pytest
import torch

import oracle
import paper_2509_23018_amd as gw
from gpu_helpers import FP64_TOL, device, rel_fro, to_dev
from workloads import gen

pytestmark = pytest.mark.gpu


def _oracle(p):
    return oracle.chi0(p.psi_v, p.psi_c, p.e_v, p.e_c, p.gvec, p.z, p.n, p.volume,
                       spin=p.spin, pair_chunk=p.pair_chunk)


def _problem(seed=61, chunk=64):
    return gen.make_problem((20, 18, 24), 5, 23, r2=15, z=(0.0, 0.6j, 0.3 + 0.01j), seed=seed,
                            pair_chunk=chunk)


@pytest.mark.parametrize("prec,ns,tol", [("fp64", 0, FP64_TOL), ("split_bf16", 5, 1e-10),
                                         ("fp32", 0, 1e-5)])
def test_chi0_in_caller_workspace(prec, ns, tol):
    """A workspace of exactly gw_workspace_bytes() bytes: same bits as the
    call with the library's scratch, and the oracle's chi."""
    p = _problem()
    dp = to_dev(p)
    kw = dict(precision=prec, n_slices=ns, pair_chunk=p.pair_chunk)
    need = gw.workspace_bytes(dp, **kw)
    assert need > 0
    ws = gw.new_workspace(need)
    got = gw.gw_chi0(dp, workspace=ws, **kw).cpu().numpy()
    ref_lib = gw.gw_chi0(to_dev(p), **kw).cpu().numpy()
    assert np.array_equal(got, ref_lib)
    assert rel_fro(got, _oracle(p)) < tol


def test_workspace_too_small_leaves_outputs():
    p = _problem(seed=62)
    dp = to_dev(p)
    need = gw.workspace_bytes(dp, pair_chunk=p.pair_chunk)
    ws = gw.new_workspace(need - 256)
    dp.chi = torch.full((len(p.z), p.ng, p.ng), 7.0 - 1.0j, dtype=torch.complex128,
                        device=device())
    with pytest.raises(gw.GWError) as ei:
        gw.gw_chi0(dp, pair_chunk=p.pair_chunk, workspace=ws)
    assert ei.value.status == -1 and "too small" in str(ei.value)
    torch.cuda.synchronize()
    assert torch.all(dp.chi == 7.0 - 1.0j)


def _batch(seed):
    out = []
    for i, (n, nv, nc, ng) in enumerate([((12, 12, 12), 3, 17, 60), ((16, 12, 14), 2, 31, 230),
                                         ((12, 12, 12), 4, 9, 140)]):
        q = np.array([0.125, -0.375, 0.375]) * (i + 1) % 1.0 - 0.5
        g = gen.gsphere_shifted(q, ng)
        nn = np.array(n)
        g = g[np.all((g >= -(nn // 2)) & (g <= (nn + 1) // 2 - 1), axis=1)]
        out.append(gen.make_problem(n, nv, nc, gvec=g, z=(0.0, 0.3j, 0.25 + 0.01j),
                                    seed=seed + 10 * i, pair_chunk=40))
    return out


@pytest.mark.parametrize("prec,ns,flags,tol", [
    ("fp64", 0, 0, FP64_TOL),
    ("fp64", 0, gw.GW_FLAG_GRAPH, FP64_TOL),
    ("split_bf16", 5, 0, 1e-10),
    ("split_bf16", 5, gw.GW_FLAG_GRAPH, 1e-10),
])
def test_batched_in_caller_workspace(prec, ns, flags, tol):
    """Several problems in one call (persistent contraction; tables staged
    into the workspace in stream order), eager and graph-captured with the
    captured work buffer in the workspace; replays with eager work between."""
    probs = _batch(seed=71)
    dps = [to_dev(p) for p in probs]
    kw = dict(precision=prec, n_slices=ns, pair_chunk=40, flags=flags)
    ws = gw.new_workspace(gw.workspace_bytes(dps, **kw))
    refs = [_oracle(p) for p in probs]
    for rep in range(3 if flags else 1):
        chis = gw.gw_chi0(dps, workspace=ws, **kw)
        torch.cuda.synchronize()
        for c, r in zip(chis, refs):
            assert rel_fro(c.cpu().numpy(), r) < tol
        torch.randn(1 << 20, device=device()).sum()
        torch.cuda.synchronize()


def test_backward_in_caller_workspace():
    p = gen.make_problem((12, 12, 12), 3, 9, r2=10, z=(0.0, 0.5j), seed=72, pair_chunk=10)
    dp = to_dev(p)
    rng = np.random.default_rng(5)
    x = rng.standard_normal((2, p.ng, p.ng)) + 1j * rng.standard_normal((2, p.ng, p.ng))
    w = np.ascontiguousarray(0.5 * (x + np.conj(np.transpose(x, (0, 2, 1)))))
    wd = torch.from_numpy(w).to(device())
    need = gw.workspace_bytes(dp, pair_chunk=p.pair_chunk, backward=True)
    ws = gw.new_workspace(need)
    got = gw.gw_chi0_backward(dp, wd, pair_chunk=p.pair_chunk, workspace=ws)
    want = oracle.chi0_backward(p.psi_v, p.psi_c, p.e_v, p.e_c, p.gvec, p.z, p.n, p.volume, w,
                                pair_chunk=p.pair_chunk)
    for g, r in zip(got, want):
        assert rel_fro(g.cpu().numpy(), r) < FP64_TOL
    with pytest.raises(gw.GWError):
        gw.gw_chi0_backward(dp, wd, pair_chunk=p.pair_chunk, workspace=ws[:need - 256])


def test_pseudobands_in_caller_workspace():
    """Tables staged without waiting: the host arrays are overwritten right
    after the call returns, before the device has run it."""
    p = gen.make_problem((12, 12, 12), 1, 40, r2=4, seed=73)
    psi = torch.from_numpy(p.psi_c).to(device())
    e = torch.from_numpy(p.e_c).to(device())
    rng = np.random.default_rng(3)
    keep, slices = np.arange(4), [np.arange(4, 20), np.arange(20, 40)]
    theta = [rng.random((3, len(s))) for s in slices]
    ws = gw.new_workspace(gw.pseudobands_workspace_bytes(4, 36, 2, 3))
    outs = []
    for rep in range(2):
        th = [t.copy() for t in theta]
        pc, ec = gw.gw_pseudobands(psi, e, keep, slices, 3, th, workspace=ws)
        for t in th:
            t[:] = 0.5            # the call must not read these any more
        outs.append((pc, ec))
    torch.cuda.synchronize()
    opc, oec = oracle.pseudobands(p.psi_c, p.e_c, keep, slices, 3, theta)
    for pc, ec in outs:
        assert np.abs(pc.cpu().numpy() - opc).max() < 1e-13 * np.abs(opc).max()
        assert np.allclose(ec.cpu().numpy(), oec, rtol=1e-15, atol=0)


def test_graph_cache_is_bounded():
    """Captured graphs beyond GW_GRAPH_CACHE_MAX are destroyed (once their
    replays are done) and their work buffers freed: device memory stays
    bounded over many distinct captured calls."""
    probs = [gen.make_problem((24, 24, 24), 4, 1000, r2=27, z=(0.2j,), seed=82),
             gen.make_problem((12, 12, 12), 3, 17, r2=9, z=(0.2j,), seed=83)]
    dps = [to_dev(p) for p in probs]
    refs = [_oracle(p) for p in probs]
    kw = dict(pair_chunk=4096, flags=gw.GW_FLAG_GRAPH)
    per_graph = gw.workspace_bytes(dps, **dict(kw, flags=0))
    assert per_graph > (128 << 20)
    outs = [[torch.empty((1, p.ng, p.ng), dtype=torch.complex128, device=device())
             for p in probs] for _ in range(8)]
    torch.cuda.synchronize()
    old = os.environ.get("GW_GRAPH_CACHE_MAX")
    os.environ["GW_GRAPH_CACHE_MAX"] = "2"
    try:
        gw.release()
        free0, _ = torch.cuda.mem_get_info()
        for k in range(8):
            for d, c in zip(dps, outs[k]):
                d.chi = c            # new output pointers: a new key, a new capture
            gw.gw_chi0(dps, **kw)
            torch.cuda.synchronize()
        gw.gw_chi0(dps, **kw)        # replay of the newest; sweeps the retired graphs
        torch.cuda.synchronize()
        free1, _ = torch.cuda.mem_get_info()
    finally:
        if old is None:
            os.environ.pop("GW_GRAPH_CACHE_MAX")
        else:
            os.environ["GW_GRAPH_CACHE_MAX"] = old
    # two cached graphs (and a few small tables) at most; eight were captured
    assert free0 - free1 <= 3 * per_graph + (64 << 20), (free0 - free1, per_graph)
    for k in (0, 7):
        for c, r in zip(outs[k], refs):
            assert rel_fro(c.cpu().numpy(), r) < FP64_TOL


def test_captured_graph_survives_plan_eviction():
    """A graph captured over two problems keeps their plans alive while more
    than 256 other plans (distinct G lists) push them out of the cache: the
    replay still matches the oracle, and so does an eager call that has to
    rebuild an evicted plan."""
    probs = _batch(seed=91)[:2]
    dps = [to_dev(p) for p in probs]
    refs = [_oracle(p) for p in probs]
    kw = dict(pair_chunk=40, flags=gw.GW_FLAG_GRAPH)
    gw.gw_chi0(dps, **kw)
    torch.cuda.synchronize()
    # 260 single-vector G lists on an 8^3 grid: 260 new plans
    q = gen.make_problem((8, 8, 8), 1, 2, gvec=np.zeros((1, 3), np.int32), seed=92)
    pv = torch.from_numpy(q.psi_v).to(device())
    pc = torch.from_numpy(q.psi_c).to(device())
    ax = np.arange(-4, 4)
    gl = np.stack(np.meshgrid(ax, ax, ax, indexing="ij"), -1).reshape(-1, 3)[:260]
    for g in gl:
        gw.gw_mtxel(pv, pc, g[None].astype(np.int32), q.n, q.volume)
    torch.cuda.synchronize()
    for d in dps:
        d.chi.zero_()
    chis = gw.gw_chi0(dps, **kw)     # replay
    torch.cuda.synchronize()
    for c, r in zip(chis, refs):
        assert rel_fro(c.cpu().numpy(), r) < FP64_TOL
    eager = gw.gw_chi0(to_dev(probs[0]), pair_chunk=40).cpu().numpy()
    assert rel_fro(eager, refs[0]) < FP64_TOL
