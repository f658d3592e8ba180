#!/usr/bin/env python3
"""Throughput of the chi0 build (MTXEL + CHI0) on one MI355X.

Workload (default): chi0 at q = 0 on a 48^3 grid (L = 10 bohr) with 64
valence x 960 conduction bands (61,440 pairs streamed in chunks of at most
4,096), the complete G-sphere |g|^2 <= 61 (2,007 vectors) and 4 real
frequencies omega in [0, 1] Ha with eta = 0.005 Ha, FP64 throughout.
Inputs are seeded synthetic orthonormal wavefunctions (no DFT data).

One step = one gw_chi0 call: every chunk's MTXEL, energy factor and CHI0
contraction for all frequencies, inputs already resident in HBM.  The JSON
line reports canonical TFLOP/s (8 N_G^2 pairs N_omega per step, the complex
GEMM count convention) and pairs/s, the roofline of the dominant kernel
(chi0_f64, FP64 MFMA) from HIP events recorded on the stream it runs on, and
the FP64 CPU oracle timed on a bounded sample of the same workload.

    python bench.py [--steps K] [--warmup W] [--no-cpu-baseline]
    python bench.py --calibrate-copy     # plain copy kernel for counter scaling
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "χ0 build TFLOP/s + pairs/s, FP64 vs split-BF16 at ≤1e-10 rel err"
FP64_PEAK_TFLOPS = 78.6      # MI355X dense FP64 (MFMA and vector)
HBM_PEAK_GBS = 8000.0
PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "chi0_f64_kernel_48cube_61440pairs_pmc.md")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2509_23018_amd", "csrc", f)
                  for f in ("chi0.hip", "common.hpp", "items.hpp")]
PROFILE_TRAFFIC_PB = os.path.join(ROOT, "profiles", "pseudo_mix_kernel_48cube_960bands_pmc.md")
KERNEL_SOURCES_PB = [os.path.join(ROOT, "paper_2509_23018_amd", "csrc", f)
                     for f in ("pseudobands.hip", "pseudobands.hpp", "common.hpp")]


def kernel_src_sha(sources=None) -> str:
    h = hashlib.sha256()
    for f in sources or KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_traffic(launch_count_per_step: int = 0, profile=None, sources=None):
    """HBM bytes per launch of a kernel from its committed counter summary
    (chi0_f64 by default), or None when the summary is missing or the
    kernel's sources changed since the counters were taken."""
    try:
        text = open(profile or PROFILE_TRAFFIC).read()
    except OSError:
        return None
    m = re.search(r"^traffic_json:\s*(\{.*\})\s*$", text, re.M)
    if not m:
        return None
    d = json.loads(m.group(1))
    if d.get("src_sha256") != kernel_src_sha(sources):
        return None
    return d.get("hbm_bytes_per_launch")


def calibrate_copy():
    import torch
    n = 1 << 27                                   # 2^27 doubles = 1 GiB per buffer
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8, "launches": 5}))


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true")
    ap.add_argument("--split-slices", type=int, nargs="*", default=[3, 4, 5],
                    help="slice counts of the split-BF16 runs (empty: none)")
    ap.add_argument("--workload", default="chi0_48cube",
                    choices=["chi0_48cube", "batched_40cube_64q", "precision_72cube",
                             "adjoint_32cube", "pseudobands_48cube"],
                    help="chi0_48cube: the contract line (default); the others print a "
                         "measurement line of their own")
    ap.add_argument("--pb-xi", type=int, default=4,
                    help="pseudobands per slice of the pseudobands_48cube workload (1..8)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the chi0 build here runs on a single MI355X "
              "(no multi-GPU path is built); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.workload == "batched_40cube_64q":
        bench_batched(args)
        return
    if args.workload == "precision_72cube":
        bench_precision(args)
        return
    if args.workload == "adjoint_32cube":
        bench_adjoint(args)
        return
    if args.workload == "pseudobands_48cube":
        bench_pseudobands(args)
        return

    import numpy as np
    import torch

    import paper_2509_23018_amd as gw
    from workloads import gen

    dev = torch.device("cuda", 0)
    t_gen = time.perf_counter()
    p = gen.make_config(1)
    print(f"[bench] inputs generated in {time.perf_counter() - t_gen:.1f} s: grid {p.n}, "
          f"{p.nv}x{p.nc} bands, {p.ng} G, {len(p.z)} frequencies", file=sys.stderr, flush=True)
    dp = gw.Chi0Problem(n=p.n, volume=p.volume,
                        psi_v=torch.from_numpy(p.psi_v).to(dev),
                        psi_c=torch.from_numpy(p.psi_c).to(dev),
                        e_v=torch.from_numpy(p.e_v).to(dev), e_c=torch.from_numpy(p.e_c).to(dev),
                        gvec=p.gvec, z=p.z)
    chunk = p.pair_chunk

    def step():
        gw.gw_chi0(dp, precision="fp64", pair_chunk=chunk)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    gw.profile_reset()
    gw.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    gw.profile_enable(False)
    n_chi, t_chi = gw.profile_read("chi0_f64")
    # the reduction of the last round's partial tiles completes the contraction
    n_tail, t_tail = gw.profile_read("chi0_tail")
    kernels = {k: gw.profile_read(k)
               for k in ("mtxel_zy", "mtxel_x", "delta", "chi0_f64", "chi0_tail")}
    gw.profile_reset()
    print(f"[bench] {args.steps} steps in {elapsed:.3f} s; per-kernel ms/step: " +
          ", ".join(f"{k} {v[1] / args.steps:.2f}" for k, v in kernels.items()),
          file=sys.stderr, flush=True)

    ng, npairs, nz = p.ng, p.npairs, len(p.z)
    flops_step = 8.0 * ng * ng * npairs * nz
    value = flops_step * args.steps / elapsed / 1e12
    pairs_s = npairs * args.steps / elapsed
    # Algorithmic work of the chi0_f64 launches: 8 flops per pair per chi entry
    # computed; a frequency with Re z = 0 has real Delta and Hermitian chi, for
    # which only the N_G (N_G + 1) / 2 entries on or above the diagonal are work.
    herm = np.real(p.z) == 0.0
    entries = float(np.sum(np.where(herm, ng * (ng + 1) / 2.0, float(ng) * ng)))
    alg_flops_step = 8.0 * npairs * entries
    launches_per_step = n_chi // max(1, args.steps)
    flops_per_launch = alg_flops_step / max(1, launches_per_step)
    avg_ms = (t_chi + t_tail) / max(1, n_chi)
    achieved = flops_per_launch / (avg_ms * 1e-3) / 1e12
    traffic = read_traffic(launches_per_step)
    # What the MFMAs execute: the default 64 x 64 tile takes each complex
    # multiply-add as three real products (6 flops, not 8) over whole tiles
    # and 16-pair stages, padding included.
    nb = -(-ng // 64)
    tiles = float(np.sum(np.where(herm, nb * (nb + 1) / 2.0, float(nb) * nb)))
    cw = max(1, min(p.nc, chunk // max(1, min(p.nv, 4))))
    vb = max(1, min(p.nv, chunk // cw))
    kcs = [min(vb, p.nv - v0) * min(cw, p.nc - c0)
           for v0 in range(0, p.nv, vb) for c0 in range(0, p.nc, cw)]
    exec_step = sum(6.0 * tiles * 64 * 64 * (-(-k // 16) * 16) for k in kcs)
    exec_per_launch = exec_step / max(1, launches_per_step)
    executed = exec_per_launch / (avg_ms * 1e-3) / 1e12

    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "chi0 at q=0, 48^3 grid, 64x960 bands (61,440 pairs, chunks of 4x960), "
                        "2,007 G, 4 real frequencies (eta 0.005 Ha), FP64",
            "grid": list(p.n), "pairs": npairs, "n_g": ng, "n_freq": nz,
            "pair_chunk": chunk, "precision": "fp64",
        },
        "pairs_per_s": round(pairs_s, 1),
        "kernel_ms_per_step": {k: round(v[1] / args.steps, 3) for k, v in kernels.items()},
        "roofline": {
            "kernel": "chi0_f64_kernel",
            "bound": "mfma",
            "achieved": round(achieved, 3),
            "peak": FP64_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": round(achieved / FP64_PEAK_TFLOPS, 4),
            "traffic": traffic,
            "launches": n_chi,
            "executed_tflops": round(executed, 3),
            "executed_frac": round(executed / FP64_PEAK_TFLOPS, 4),
            "executed_flops_per_launch": exec_per_launch,
            "avg_launch_ms": round(avg_ms, 4),
            "tail_reduce_ms_per_launch": round(t_tail / max(1, n_chi), 4),
            "flops_per_launch": flops_per_launch,
        },
    }

    # split-BF16 contraction on the same workload: the FP64 chi above is the
    # reference for its error (FP64 parity with the oracle is tested separately)
    ref = gw.gw_chi0(dp, precision="fp64", pair_chunk=chunk).clone()
    splits = []
    for ns in args.split_slices:
        def sstep():
            gw.gw_chi0(dp, precision="split_bf16", n_slices=ns, pair_chunk=chunk)
        sstep()
        torch.cuda.synchronize()
        gw.profile_reset()
        gw.profile_enable(True)
        t0 = time.perf_counter()
        for _ in range(args.steps):
            sstep()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        gw.profile_enable(False)
        ks = {k: gw.profile_read(k)
              for k in ("mtxel_zy", "mtxel_x", "split_prep", "chi0_split", "chi0_split_tail")}
        gw.profile_reset()
        got = dp.chi
        err = float(torch.linalg.vector_norm(got - ref) / torch.linalg.vector_norm(ref))
        splits.append({
            "n_slices": ns,
            "value": round(flops_step * args.steps / el / 1e12, 3),
            "unit": "TFLOP/s",
            "pairs_per_s": round(npairs * args.steps / el, 1),
            "ms_per_step": round(el / args.steps * 1e3, 3),
            "speedup_vs_fp64": round(elapsed / el, 3),
            "rel_err_vs_fp64": err,
            "kernel_ms_per_step": {k: round(v[1] / args.steps, 3) for k, v in ks.items()},
        })
        print(f"[bench] split_bf16 S={ns}: {el / args.steps * 1e3:.1f} ms/step, rel err {err:.2e}",
              file=sys.stderr, flush=True)
    out["split_bf16"] = splits
    ok = [x for x in splits if x["rel_err_vs_fp64"] <= 1e-10]
    out["split_bf16_at_1e-10"] = min(ok, key=lambda x: x["n_slices"]) if ok else None
    dp.chi = None

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(p, dp, dev)
    print(json.dumps(out), flush=True)


def _timed(fn, steps):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def bench_batched(args):
    """64 q-points (4x4x4 shifted grid) on a 40^3 grid, 48 valence bands and
    300-900 conduction bands each, G-spheres of 400-4,000 vectors, 16
    imaginary frequencies: one graph-captured gw_chi0 call over all problems,
    FP64 and split BF16.  Band sets are drawn on the GPU (timing only; parity
    of this workload is tested on four q-points at full size)."""
    import numpy as np
    import torch

    import paper_2509_23018_amd as gw
    from workloads import gen

    dev = torch.device("cuda", 0)
    qs, ngs, ncs = gen.batched_shapes()
    z = gen.frequencies("imag", 16)
    n, nv = (40, 40, 40), 48
    nr = int(np.prod(n))
    volume = gen.CELL_L ** 3
    t_gen = time.perf_counter()
    probs, flops, pairs = [], 0.0, 0
    for qi in range(qs.shape[0]):
        nc, ng = int(ncs[qi]), int(ngs[qi])
        rng = np.random.default_rng(4000 + qi)
        e_v, e_c = gen.band_energies(rng, nv, nc)
        psi = gen.device_bands(nv + nc, nr, seed=4000 + qi, volume=volume, device=dev)
        probs.append(gw.Chi0Problem(n=n, volume=volume, psi_v=psi[:nv], psi_c=psi[nv:],
                                    e_v=torch.from_numpy(e_v).to(dev),
                                    e_c=torch.from_numpy(e_c).to(dev),
                                    gvec=gen.gsphere_shifted(qs[qi], ng), z=z))
        flops += 8.0 * ng * ng * nv * nc * len(z)
        pairs += nv * nc
    torch.cuda.synchronize()
    torch.cuda.empty_cache()  # hand cached blocks back: the library allocates outside torch
    free, total = torch.cuda.mem_get_info()
    print(f"[bench] device memory free {free / 2**30:.1f} of {total / 2**30:.1f} GiB",
          file=sys.stderr, flush=True)
    print(f"[bench] 64 problems generated in {time.perf_counter() - t_gen:.1f} s "
          f"({pairs} pairs, {flops:.3e} canonical flops per call)", file=sys.stderr, flush=True)
    out = {"workload": "batched_40cube_64q", "problems": len(probs), "pairs": pairs,
           "n_freq": len(z), "canonical_flops": flops, "data": "synthetic (device Gaussian bands)",
           "runs": []}
    ref = None
    keep = [int(np.argmin(ngs)), int(np.argmax(ngs)), int(np.argmax(ncs))]
    for prec, ns in [("fp64", 0)] + [("split_bf16", k) for k in args.split_slices]:
        def call():
            gw.gw_chi0(probs, precision=prec, n_slices=ns, flags=gw.GW_FLAG_GRAPH)
        t_cap = time.perf_counter()
        call()  # builds plans, captures the graph, runs once
        torch.cuda.synchronize()
        t_cap = time.perf_counter() - t_cap
        gw.profile_reset()
        gw.profile_enable(True)
        dt = _timed(call, max(1, args.steps))
        gw.profile_enable(False)
        gw.profile_reset()
        run = {"precision": prec, "n_slices": ns or None, "s_per_call": round(dt, 4),
               "first_call_s": round(t_cap, 3), "tflops": round(flops / dt / 1e12, 3),
               "pairs_per_s": round(pairs / dt, 1)}
        if prec == "fp64":
            ref = [probs[q].chi.clone() for q in keep]
        else:
            num = sum(float(torch.linalg.vector_norm(probs[q].chi - r) ** 2) for q, r in zip(keep, ref))
            den = sum(float(torch.linalg.vector_norm(r) ** 2) for r in ref)
            run["rel_err_vs_fp64"] = (num / den) ** 0.5
            run["speedup_vs_fp64"] = round(out["runs"][0]["s_per_call"] / dt, 3)
        out["runs"].append(run)
        free, total = torch.cuda.mem_get_info()
        print(f"[bench] batched {prec} S={ns}: {dt:.3f} s per call; device memory free "
              f"{free / 2**30:.1f} of {total / 2**30:.1f} GiB, torch reserved "
              f"{torch.cuda.memory_reserved() / 2**30:.1f} GiB", file=sys.stderr, flush=True)
    out["err_sample_q"] = keep
    gw.release()
    print(json.dumps(out), flush=True)


def bench_precision(args):
    """chi0 on a 72^3 grid, 256 x 3,840 bands (983,040 pairs), 6,031 G, 8
    imaginary frequencies, in FP64, FP32 and split BF16; errors against the
    FP64 result on the 32 G rows drawn with seed 1002.  Band sets are drawn
    on the GPU (timing only)."""
    import numpy as np
    import torch

    import paper_2509_23018_amd as gw
    from workloads import gen

    dev = torch.device("cuda", 0)
    sh = gen.CONFIG_SHAPES[2]
    n, nv, nc = sh["n"], sh["nv"], sh["nc"]
    nr = int(np.prod(n))
    volume = gen.CELL_L ** 3
    z = gen.frequencies(*sh["freq"])
    gvec = gen.gsphere(sh["r2"])
    rng = np.random.default_rng(2)
    e_v, e_c = gen.band_energies(rng, nv, nc)
    psi = gen.device_bands(nv + nc, nr, seed=2, volume=volume, device=dev)
    torch.cuda.empty_cache()
    ng = gvec.shape[0]
    rows = np.sort(np.random.default_rng(1002).choice(ng, 32, replace=False))
    flops = 8.0 * ng * ng * nv * nc * len(z)
    prob = gw.Chi0Problem(n=n, volume=volume, psi_v=psi[:nv], psi_c=psi[nv:],
                          e_v=torch.from_numpy(e_v).to(dev), e_c=torch.from_numpy(e_c).to(dev),
                          gvec=gvec, z=z)
    # plans and tables of this grid and G list, built outside the timed calls
    warm = gw.Chi0Problem(n=n, volume=volume, psi_v=psi[:1], psi_c=psi[nv:nv + 64],
                          e_v=prob.e_v[:1], e_c=prob.e_c[:64], gvec=gvec, z=z)
    out = {"workload": "precision_72cube", "pairs": nv * nc, "n_g": ng, "n_freq": len(z),
           "canonical_flops": flops, "data": "synthetic (device Gaussian bands)",
           "err_rows": "32 rows, numpy default_rng(1002)", "runs": []}
    ref = None
    modes = [("fp64", 0), ("fp32", 0)] + [("split_bf16", k) for k in args.split_slices]
    for prec, ns in modes:
        gw.gw_chi0(warm, precision=prec, n_slices=ns)
        torch.cuda.synchronize()
        dt = _timed(lambda: gw.gw_chi0(prob, precision=prec, n_slices=ns), 1)
        sub = prob.chi[:, torch.from_numpy(rows).to(dev)].clone()
        run = {"precision": prec, "n_slices": ns or None, "s_per_call": round(dt, 3),
               "tflops": round(flops / dt / 1e12, 3), "pairs_per_s": round(nv * nc / dt, 1)}
        if prec == "fp64":
            ref = sub
        else:
            run["rel_err_vs_fp64"] = float(torch.linalg.vector_norm(sub - ref) /
                                           torch.linalg.vector_norm(ref))
            run["rel_err_per_freq"] = [float(torch.linalg.vector_norm(sub[w] - ref[w]) /
                                             torch.linalg.vector_norm(ref[w]))
                                       for w in range(len(z))]
            run["speedup_vs_fp64"] = round(out["runs"][0]["s_per_call"] / dt, 3)
        out["runs"].append(run)
        print(f"[bench] precision {prec} S={ns}: {dt:.2f} s", file=sys.stderr, flush=True)
    gw.release()
    print(json.dumps(out), flush=True)


ADJOINT_KERNELS = ("mtxel_zy", "mtxel_x", "delta", "bwd_gm", "bwd_de", "bwd_de_reduce", "bwd_x",
                   "bwd_yz", "bwd_reduce_cv", "bwd_reduce_c", "bwd_reduce_v")


def bench_adjoint(args):
    """The adjoint of chi0 (gw_chi0_backward) on the 32^3 workload: 32 x 480
    bands (15,360 pairs), 1,189 G, static; grad_chi = A, a seeded Hermitian
    matrix with N(0,1) entries (the gradient of L = Re tr(A chi)).  Times the
    forward call and the adjoint, per kernel, and the oracle adjoint on a
    bounded sample of the same workload (8 of 32 valence bands) on the host."""
    import numpy as np
    import torch

    import paper_2509_23018_amd as gw
    from workloads import gen

    dev = torch.device("cuda", 0)
    t_gen = time.perf_counter()
    p = gen.make_config(3)
    rng = np.random.default_rng(1003)
    x = rng.standard_normal((p.ng, p.ng)) + 1j * rng.standard_normal((p.ng, p.ng))
    a_np = 0.5 * (x + x.conj().T)
    w = torch.from_numpy(a_np[None].copy()).to(dev)

    def to_dev(q):
        return gw.Chi0Problem(n=q.n, volume=q.volume, psi_v=torch.from_numpy(q.psi_v).to(dev),
                              psi_c=torch.from_numpy(q.psi_c).to(dev),
                              e_v=torch.from_numpy(q.e_v).to(dev),
                              e_c=torch.from_numpy(q.e_c).to(dev), gvec=q.gvec, z=q.z)

    dp = to_dev(p)
    torch.cuda.synchronize()
    print(f"[bench] adjoint inputs generated in {time.perf_counter() - t_gen:.1f} s: grid {p.n}, "
          f"{p.nv}x{p.nc} bands, {p.ng} G", file=sys.stderr, flush=True)
    ng, npairs, nz = p.ng, p.npairs, len(p.z)
    chunk = p.pair_chunk

    def fwd():
        gw.gw_chi0(dp, precision="fp64", pair_chunk=chunk)

    def bwd():
        gw.gw_chi0_backward(dp, w, pair_chunk=chunk)

    for _ in range(max(1, args.warmup)):
        fwd()
        bwd()
    torch.cuda.synchronize()
    steps = max(1, args.steps)
    t_fwd = _timed(fwd, steps)
    gw.profile_reset()
    gw.profile_enable(True)
    t_bwd = _timed(bwd, steps)
    gw.profile_enable(False)
    kernels = {k: gw.profile_read(k) for k in ADJOINT_KERNELS}
    gw.profile_reset()
    # The adjoint's GEMMs P1 = M W and P2 = M W^H: 2 x 8 flops per (pair, G, G')
    # per frequency, twice the forward contraction.
    gemm_flops = 2.0 * 8.0 * npairs * ng * ng * nz
    n_gm, t_gm = kernels["bwd_gm"]
    gm_per_launch = gemm_flops / max(1, n_gm // steps)
    gm_avg_ms = t_gm / max(1, n_gm)
    achieved = gm_per_launch / (gm_avg_ms * 1e-3) / 1e12
    out = {
        "workload": "adjoint_32cube",
        "config": {"grid": list(p.n), "pairs": npairs, "n_g": ng, "n_freq": nz,
                   "pair_chunk": chunk, "precision": "fp64",
                   "grad_chi": "seeded Hermitian N(0,1) matrix (seed 1003)"},
        "data": "synthetic",
        "s_per_forward": round(t_fwd, 5),
        "s_per_adjoint": round(t_bwd, 5),
        "adjoint_over_forward": round(t_bwd / t_fwd, 3),
        "adjoint_gemm_tflops_per_s": round(gemm_flops / t_bwd / 1e12, 3),
        "pairs_per_s": round(npairs / t_bwd, 1),
        "kernel_ms_per_call": {k: round(v[1] / steps, 3) for k, v in kernels.items()},
        "roofline": {
            "kernel": "bwd_gm_kernel",
            "bound": "mfma",
            "achieved": round(achieved, 3),
            "peak": FP64_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": round(achieved / FP64_PEAK_TFLOPS, 4),
            "traffic": None,
            "launches": n_gm,
            "avg_launch_ms": round(gm_avg_ms, 4),
            "flops_per_launch": gm_per_launch,
        },
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_adjoint(p, a_np, dev)
    gw.release()
    print(json.dumps(out), flush=True)


PB_SIZES = [16, 32, 64, 128, 256, 400]   # slices of the 896 unprotected conduction bands
PB_PROTECT = 64


def bench_pseudobands(args):
    """Stochastic pseudobands on workload 1 (48^3 grid, 64 x 960 bands, 2,007 G,
    4 real frequencies): the 64 lowest conduction bands are protected and the
    other 896 become n_xi pseudobands (4 by default) per slice of 16, 32, 64, 128, 256 and 400
    bands (88 conduction bands in all at n_xi = 4), then chi0 is built in FP64 on the
    compressed set.  Reports the mixing kernel against the HBM roofline, the
    chi0 time and its error against chi0 on all 960 bands, and the oracle's
    pseudobands timed on the host."""
    import numpy as np
    import torch

    import paper_2509_23018_amd as gw
    from workloads import gen

    dev = torch.device("cuda", 0)
    xi = args.pb_xi
    p = gen.make_config(1)
    keep, slices, theta = gen.pseudoband_recipe(p.e_c, PB_PROTECT, PB_SIZES, xi, seed=1005)
    chunk = p.pair_chunk

    def prob(psi_c, e_c):
        return gw.Chi0Problem(n=p.n, volume=p.volume, psi_v=torch.from_numpy(p.psi_v).to(dev),
                              psi_c=psi_c, e_v=torch.from_numpy(p.e_v).to(dev), e_c=e_c,
                              gvec=p.gvec, z=p.z)

    pc_full = torch.from_numpy(p.psi_c).to(dev)
    ec_full = torch.from_numpy(p.e_c).to(dev)
    full = gw.gw_chi0(prob(pc_full, ec_full), precision="fp64", pair_chunk=chunk)
    t_full = _timed(lambda: gw.gw_chi0(prob(pc_full, ec_full), precision="fp64",
                                       pair_chunk=chunk), max(1, args.steps))

    def make_pb():
        return gw.gw_pseudobands(pc_full, ec_full, keep, slices, xi, theta)

    for _ in range(max(1, args.warmup)):
        make_pb()
    steps = max(1, args.steps)
    gw.profile_reset()
    gw.profile_enable(True)
    t_pb = _timed(make_pb, steps)
    gw.profile_enable(False)
    n_mix, t_mix = gw.profile_read("pseudo_mix")
    n_keep, t_keep = gw.profile_read("pseudo_keep")
    n_prep, t_prep = gw.profile_read("pseudo_prep")
    gw.profile_reset()
    pc, ec = make_pb()
    dq = prob(pc, ec)
    chi_c = gw.gw_chi0(dq, precision="fp64", pair_chunk=chunk)
    t_chi = _timed(lambda: gw.gw_chi0(dq, precision="fp64", pair_chunk=chunk), steps)
    diff = (chi_c - full).cpu().numpy()
    ref = full.cpu().numpy()
    err = float(np.linalg.norm(diff) / np.linalg.norm(ref))
    err_w = [float(np.linalg.norm(diff[w]) / np.linalg.norm(ref[w])) for w in range(len(p.z))]
    # the diagonal and the trace keep their expectation term by term (the
    # cross terms of a slice average out there); off-diagonal entries of
    # white-noise bands do not decay, so their stochastic error is of the
    # order of the entries themselves
    dg_c = np.diagonal(chi_c.cpu().numpy(), axis1=1, axis2=2)
    dg_f = np.diagonal(ref, axis1=1, axis2=2)
    err_diag = [float(np.linalg.norm(dg_c[w] - dg_f[w]) / np.linalg.norm(dg_f[w]))
                for w in range(len(p.z))]
    err_trace = [float(abs(dg_c[w].sum() - dg_f[w].sum()) / abs(dg_f[w].sum()))
                 for w in range(len(p.z))]
    nr = int(np.prod(p.n))
    nmixed = sum(len(s) for s in slices)
    # algorithmic bytes of one mixing launch: every slice band read once, the
    # pseudobands written once
    mix_bytes = 16.0 * nr * (nmixed + len(slices) * xi)
    mix_ms = t_mix / max(1, n_mix)
    achieved = mix_bytes / (mix_ms * 1e-3) / 1e9
    nc_out = PB_PROTECT + len(slices) * xi
    out = {
        "workload": "pseudobands_48cube",
        "config": {"grid": list(p.n), "n_v": p.nv, "n_c": p.nc, "n_g": p.ng,
                   "n_freq": len(p.z), "protected": PB_PROTECT, "slices": PB_SIZES,
                   "n_xi": xi, "n_c_compressed": nc_out, "theta_seed": 1005},
        "data": "synthetic",
        "s_per_pseudobands": round(t_pb, 5),
        "pseudo_mix_ms": round(mix_ms, 4),
        "pseudo_keep_ms": round(t_keep / max(1, n_keep), 4),
        "pseudo_prep_ms": round(t_prep / max(1, n_prep), 4),
        "s_per_chi0_compressed": round(t_chi, 5),
        "s_per_chi0_full": round(t_full, 5),
        "speedup_chi0": round(t_full / (t_chi + t_pb), 3),
        "rel_err_vs_full": err,
        "rel_err_per_freq": err_w,
        "rel_err_diagonal_per_freq": err_diag,
        "rel_err_trace_per_freq": err_trace,
        "roofline": {
            "kernel": "pseudo_mix_kernel",
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": read_traffic(profile=PROFILE_TRAFFIC_PB, sources=KERNEL_SOURCES_PB),
            "launches": n_mix,
            "avg_launch_ms": round(mix_ms, 4),
            "bytes_per_launch": mix_bytes,
        },
    }
    if not args.no_cpu_baseline:
        import oracle
        t0 = time.perf_counter()
        opc, oec = oracle.pseudobands(p.psi_c, p.e_c, keep, slices, xi, theta)
        dt = time.perf_counter() - t0
        dev_err = float(np.abs(pc.cpu().numpy() - opc).max() / np.abs(opc).max())
        out["cpu_baseline"] = {"value": round(mix_bytes / dt / 1e9, 2), "unit": "GB/s",
                               "cores": 1, "kind": "oracle",
                               "sample": "the whole compression (all slices), numpy",
                               "seconds": round(dt, 2), "gpu_max_rel_diff": dev_err}
    gw.release()
    print(json.dumps(out), flush=True)


def cpu_baseline_adjoint(p, a_np, dev):
    """The FP64 oracle adjoint on a bounded sample: the first eight valence
    bands against all conduction bands (3,840 pairs, about 10-15 s), timed on
    this host; the device adjoint of the same sample is compared with it."""
    import numpy as np
    import torch

    import oracle
    import paper_2509_23018_amd as gw

    try:
        from threadpoolctl import threadpool_info
        blas_threads = max([i.get("num_threads", 1) for i in threadpool_info()
                            if i.get("user_api") == "blas"] or [1])
    except Exception:  # threadpoolctl missing: report the process's CPU count
        blas_threads = os.cpu_count() or 1
    nvs = 8
    t0 = time.perf_counter()
    ref = oracle.chi0_backward(p.psi_v[:nvs], p.psi_c, p.e_v[:nvs], p.e_c, p.gvec, p.z, p.n,
                               p.volume, a_np[None], spin=p.spin)
    dt = time.perf_counter() - t0
    sub = gw.Chi0Problem(n=p.n, volume=p.volume, psi_v=torch.from_numpy(p.psi_v[:nvs]).to(dev),
                         psi_c=torch.from_numpy(p.psi_c).to(dev),
                         e_v=torch.from_numpy(p.e_v[:nvs]).to(dev),
                         e_c=torch.from_numpy(p.e_c).to(dev), gvec=p.gvec, z=p.z)
    got = gw.gw_chi0_backward(sub, torch.from_numpy(a_np[None].copy()).to(dev),
                              pair_chunk=p.pair_chunk)
    num = sum(float(np.linalg.norm(g.cpu().numpy() - r) ** 2) for g, r in zip(got, ref))
    den = sum(float(np.linalg.norm(r) ** 2) for r in ref)
    pairs = nvs * p.nc
    return {"value": round(pairs / dt, 1), "unit": "pairs/s", "cores": blas_threads,
            "kind": "oracle",
            "sample": f"{nvs} of {p.nv} valence bands x all {p.nc} conduction bands ({pairs} of "
                      f"{p.npairs} pairs), all {p.ng} G; numpy FFTs per pair + BLAS",
            "seconds": round(dt, 2), "gpu_rel_err_on_sample": (num / den) ** 0.5}


def cpu_baseline(p, dp, dev):
    """The FP64 oracle on a bounded sample of the workload: the first eight
    valence bands against all conduction bands (7,680 pairs, about 10 s on 16
    cores), every G and frequency, timed on this host; the device result for
    the same sample is compared with it."""
    import numpy as np
    import torch

    import oracle
    import paper_2509_23018_amd as gw

    try:
        from threadpoolctl import threadpool_info
        blas_threads = max([i.get("num_threads", 1) for i in threadpool_info()
                            if i.get("user_api") == "blas"] or [1])
    except Exception:  # pragma: no cover
        blas_threads = os.cpu_count() or 1
    nv_s = 8
    t0 = time.perf_counter()
    ref = oracle.chi0(p.psi_v[:nv_s], p.psi_c, p.e_v[:nv_s], p.e_c, p.gvec, p.z, p.n, p.volume,
                      spin=p.spin, pair_chunk=p.pair_chunk)
    dt = time.perf_counter() - t0
    sub = gw.Chi0Problem(n=p.n, volume=p.volume, psi_v=dp.psi_v[:nv_s].contiguous(),
                         psi_c=dp.psi_c, e_v=dp.e_v[:nv_s].contiguous(), e_c=dp.e_c,
                         gvec=p.gvec, z=p.z)
    got = gw.gw_chi0(sub, pair_chunk=p.pair_chunk).cpu().numpy()
    err = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    pairs = nv_s * p.nc
    flops = 8.0 * p.ng * p.ng * pairs * len(p.z)
    return {
        "value": round(flops / dt / 1e12, 5),
        "unit": "TFLOP/s",
        "cores": int(blas_threads),
        "kind": "oracle",
        "sample": f"{nv_s} of {p.nv} valence bands x all {p.nc} conduction bands "
                  f"({pairs} of {p.npairs} pairs), all {p.ng} G and {len(p.z)} frequencies; "
                  "numpy FFT per pair (one thread) + BLAS contraction",
        "seconds": round(dt, 2),
        "pairs_per_s": round(pairs / dt, 2),
        "gpu_rel_err_on_sample": err,
    }


if __name__ == "__main__":
    main()
