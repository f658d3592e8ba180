"""The two LDS rings of the split contractions (one or two k-steps per ring
stage, at the depth each fits) and the autotuner that picks between them.

A ring only changes when a k-step's slices land in LDS, not which MFMAs
consume them or in what order, so every ring must give the same bits; the
autotuner times both on the first chunk into scratch and must leave the
result bit-identical to an untuned call."""
import os

import numpy as np
import pytest
import torch

import oracle
import paper_2509_23018_amd as gw
from gpu_helpers import rel_fro, run_chi0, to_dev
from workloads import gen

pytestmark = pytest.mark.gpu


def _with_ring(v, fn):
    os.environ["GW_SPLIT_VARIANT"] = str(v)
    try:
        return fn()
    finally:
        os.environ.pop("GW_SPLIT_VARIANT", None)


# 6 x 120 = 720 pairs in chunks of 600: two chunks, several 128-pair blocks
# and a ragged last block; few tiles, so the last round is cut into parts
@pytest.mark.parametrize("prec,S", [("split_bf16", 2), ("split_bf16", 3), ("split_bf16", 4),
                                    ("split_bf16", 5), ("split_bf16", 6),
                                    ("split_fp16x9", 3), ("split_fp16x9", 4)])
def test_split_rings_same_bits(prec, S):
    p = gen.make_problem((16, 14, 18), 6, 120, r2=12, z=(0.0, 0.3j, 0.2 + 0.01j), seed=61,
                         pair_chunk=600)
    a = _with_ring(0, lambda: run_chi0(p, precision=prec, n_slices=S))
    b = _with_ring(1, lambda: run_chi0(p, precision=prec, n_slices=S))
    assert np.array_equal(a, b), (prec, S, rel_fro(a, b))
    if S >= 5:
        ref = oracle.chi0(p.psi_v, p.psi_c, p.e_v, p.e_c, p.gvec, p.z, p.n, p.volume,
                          spin=p.spin, pair_chunk=p.pair_chunk)
        assert rel_fro(a, ref) <= 1e-10


@pytest.mark.parametrize("S", [3, 5])
def test_batched_split_rings_same_bits(S):
    probs = [gen.make_problem((14, 12, 16), 4, nc, r2=r2, z=(0.0, 0.25j), seed=70 + i,
                              pair_chunk=200)
             for i, (nc, r2) in enumerate([(50, 9), (90, 14), (30, 6)])]
    outs = []
    for v in (0, 1):
        def run():
            dps = [to_dev(p) for p in probs]
            chis = gw.gw_chi0(dps, precision="split_bf16", n_slices=S, pair_chunk=200)
            torch.cuda.synchronize()
            return [c.cpu().numpy() for c in chis]
        outs.append(_with_ring(v, run))
    for a, b in zip(*outs):
        assert np.array_equal(a, b)


def test_split_autotune_same_bits_and_cache(tmp_path):
    cache = tmp_path / "tune.txt"
    os.environ["GW_AUTOTUNE_CACHE"] = str(cache)
    try:
        p = gen.make_problem((18, 16, 14), 5, 77, r2=13, z=(0.0, 0.5j), seed=81, pair_chunk=300)
        want = run_chi0(p, precision="split_bf16", n_slices=4)
        got = run_chi0(p, precision="split_bf16", n_slices=4, flags=gw.GW_FLAG_AUTOTUNE)
        assert np.array_equal(got, want)
        # a batch of two problems of other shapes tunes the batched ring on
        # the larger one; each result equals its one-problem call
        qs = [gen.make_problem((18, 16, 14), 5, nc, r2=r2, z=(0.0, 0.5j), seed=82 + i,
                              pair_chunk=300) for i, (nc, r2) in enumerate([(61, 11), (40, 7)])]
        got_b = [c.cpu().numpy() for c in
                 gw.gw_chi0([to_dev(q) for q in qs], precision="split_bf16", n_slices=3,
                            pair_chunk=300, flags=gw.GW_FLAG_AUTOTUNE)]
        for q, g in zip(qs, got_b):
            assert np.array_equal(g, run_chi0(q, precision="split_bf16", n_slices=3))
    finally:
        os.environ.pop("GW_AUTOTUNE_CACHE", None)
    lines = [ln.split() for ln in cache.read_text().splitlines() if ln.strip()]
    kinds = {ln[0] for ln in lines}
    assert {"sbf16-S4", "sbf16-S3"} <= kinds, lines
    for ln in lines:
        assert int(ln[3]) in (0, 1) and len(ln) == 4 + 2, ln   # variant and two timings
