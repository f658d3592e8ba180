#!/usr/bin/env python3
"""Throughput of the chi0 build (MTXEL + CHI0) on one MI355X.

Contract workload (default, ``--workload chi0_72cube``): the precision study
of chi0 at q = 0 on a 72^3 grid (L = 10 bohr) with 256 valence x 3,840
conduction bands (983,040 pairs), the complete G-sphere |g|^2 <= 126 (6,031
vectors) and 8 imaginary frequencies on a Gauss-Legendre grid.  Inputs are
seeded Gaussian wavefunctions orthonormalised on the grid (no DFT data).

One step = one gw_chi0 call over one NV block (16 valence bands x all
conduction bands, 61,440 pairs, streamed in chunks of 4 x 1,024 pairs)
accumulated into the full chi with the Hermitian shortcut kept; 16 steps
build the whole chi0, inputs already resident in HBM.  The JSON line reports
canonical TFLOP/s (8 N_G^2 pairs N_omega per step, the complex GEMM count
convention) and pairs/s, the roofline of the dominant kernel (chi0_f64, FP64
MFMA, executed flops) from HIP events recorded on the stream it runs on,
MTXEL's share and rate, one whole build in FP64, FP32 and split BF16 with
errors against the device FP64 build (32 rows), every precision on a
4 x 512-band sample against the FP64 oracle, and the oracle's time on that
sample (the CPU baseline).

    python bench.py [--steps K] [--warmup W] [--no-cpu-baseline] [--no-legs]
    python bench.py --workload {chi0_48cube,batched_40cube_64q,adjoint_32cube,
                                pseudobands_48cube}
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
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-legs", action="store_true",
                    help="chi0_72cube: time FP64 only (no FP32 / split legs, no error sample)")
    ap.add_argument("--calibrate-copy", action="store_true")
    ap.add_argument("--profile-inputs", action="store_true",
                    help="chi0_72cube: Gaussian bands drawn on the device, not orthonormalised "
                         "(counter runs only: the work does not depend on the values)")
    ap.add_argument("--split-slices", type=int, nargs="*", default=None,
                    help="slice counts of the split-BF16 runs (default 3 4 5; empty: none)")
    ap.add_argument("--workload", default="chi0_72cube",
                    choices=["chi0_72cube", "chi0_48cube", "batched_40cube_64q",
                             "adjoint_32cube", "pseudobands_48cube", "subspace_72cube",
                             "epsinv_72cube", "gpp_offdiag"],
                    help="chi0_72cube: the contract line (default); the others print a "
                         "measurement line of their own")
    ap.add_argument("--pb-xi", type=int, default=4,
                    help="pseudobands per slice of the pseudobands_48cube workload (1..8)")
    args = ap.parse_args()
    if args.split_slices is None:
        args.split_slices = [3, 4, 5]
    if args.gpus != 1:
        print("bench.py measures one GPU: the chi0 build here runs on a single MI355X "
              "(no multi-GPU path is built); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.calibrate_copy:
        calibrate_copy()
        return
    {"chi0_72cube": bench_chi0_72cube, "chi0_48cube": bench_chi0_48cube,
     "batched_40cube_64q": bench_batched, "adjoint_32cube": bench_adjoint,
     "pseudobands_48cube": bench_pseudobands, "subspace_72cube": bench_subspace,
     "epsinv_72cube": bench_epsinv, "gpp_offdiag": bench_gpp}[args.workload](args)


W2_BLOCK_NV = 16        # valence bands per step of the 72^3 workload (one NV block)
W2_SAMPLE = (4, 512)    # valence x conduction bands of its oracle sample
PROFILE_TRAFFIC_72 = os.path.join(ROOT, "profiles", "chi0_f64_kernel_72cube_983040pairs_pmc.md")


def _log(t_start, msg):
    print(f"[bench +{time.perf_counter() - t_start:6.1f} s] {msg}", file=sys.stderr, flush=True)


def host_info():
    """Cores this process may use, the CPU model and the BLAS numpy calls."""
    info = {"cores_available": len(os.sched_getaffinity(0)), "cpu_model": None, "blas": None,
            "blas_threads": None}
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    info["cpu_model"] = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        from threadpoolctl import threadpool_info
        blas = [i for i in threadpool_info() if i.get("user_api") == "blas"]
        if blas:
            info["blas"] = f"{blas[0].get('internal_api')} {blas[0].get('version')}"
            info["blas_threads"] = max(int(i.get("num_threads", 1)) for i in blas)
    except Exception:
        pass
    return info


def chunk_pairs(nv, nc, chunk):
    """Pairs of each streamed chunk: the library cuts the pairs into rectangles
    of vb valence x cw conduction bands (at least 4 valence bands high)."""
    cw = max(1, min(nc, chunk // max(1, min(nv, 4))))
    vb = max(1, min(nv, chunk // cw))
    return [min(vb, nv - v0) * min(cw, nc - c0)
            for v0 in range(0, nv, vb) for c0 in range(0, nc, cw)]


def f64_flops(kcs, ng, herm):
    """(executed, algorithmic) flops of the chi0_f64 launches over chunks of
    kcs pairs.  Executed: the default 64x64 tile takes a complex multiply-add
    as three real MFMA products (6 flops) over whole tiles and 16-pair stages;
    algorithmic: 8 flops per (pair, entry), a Hermitian frequency counting the
    N_G (N_G + 1) / 2 entries on or above the diagonal."""
    import numpy as np
    herm = np.asarray(herm, bool)
    nb = -(-ng // 64)
    tiles = float(np.sum(np.where(herm, nb * (nb + 1) / 2.0, float(nb) * nb)))
    entries = float(np.sum(np.where(herm, ng * (ng + 1) / 2.0, float(ng) * ng)))
    executed = sum(6.0 * tiles * 64 * 64 * (-(-k // 16) * 16) for k in kcs)
    algorithmic = sum(8.0 * k * entries for k in kcs)
    return executed, algorithmic


def bench_chi0_72cube(args):
    """The contract line: chi0 of the 72^3 precision-study workload (256 x 3,840
    bands = 983,040 pairs, 6,031 G, 8 imaginary frequencies), seeded recipe
    bands orthonormalised on the device.  One step = one gw_chi0 call over one
    NV block of 16 valence bands x all 3,840 conduction bands (61,440 pairs,
    16 chunks of at most 4 x 1,024), accumulated into the full chi (the first
    block of every cycle overwrites it): 16 steps build the whole chi0.  Also
    times one whole build in FP64, FP32 and split BF16 (3, 4, 5 slices) with
    their 32-row errors against the device FP64 build, and every precision on
    a 4 x 512-band sample against the FP64 oracle, which is the CPU baseline."""
    import numpy as np
    import torch

    import paper_2509_23018_amd as gw
    from workloads import gen

    t_start = time.perf_counter()
    dev = torch.device("cuda", 0)
    if args.profile_inputs:
        sh = gen.CONFIG_SHAPES[2]
        rng = np.random.default_rng(2)
        e_v, e_c = gen.band_energies(rng, sh["nv"], sh["nc"])
        w = gen.DeviceProblem(n=sh["n"], volume=gen.CELL_L ** 3,
                              psi=gen.device_bands(sh["nv"] + sh["nc"], int(np.prod(sh["n"])),
                                                   seed=2, device=dev),
                              nv=sh["nv"], e_v=e_v, e_c=e_c, gvec=gen.gsphere(sh["r2"]),
                              z=gen.frequencies(*sh["freq"]), pair_chunk=sh["pair_chunk"])
    else:
        w = gen.make_config_device(2, device=dev)
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    n, nv, nc, ng, nz = w.n, w.nv, w.nc, w.ng, len(w.z)
    _log(t_start, f"inputs ready: grid {n}, {nv}x{nc} recipe bands (orthonormalised on the "
                  f"device), {ng} G, {nz} imaginary frequencies")
    ev_d = torch.from_numpy(w.e_v).to(dev)
    ec_d = torch.from_numpy(w.e_c).to(dev)
    vbk = W2_BLOCK_NV
    nblk = nv // vbk
    chi = torch.empty((nz, ng, ng), dtype=torch.complex128, device=dev)
    psi_c = w.psi_c
    probs = [gw.Chi0Problem(n=n, volume=w.volume, psi_v=w.psi[b * vbk:(b + 1) * vbk],
                            psi_c=psi_c, e_v=ev_d[b * vbk:(b + 1) * vbk], e_c=ec_d,
                            gvec=w.gvec, z=w.z, chi=chi) for b in range(nblk)]
    acc = gw.GW_FLAG_ACCUMULATE | gw.GW_FLAG_ACC_HERMITIAN

    def step(k, prec="fp64", ns=0, extra=0):
        b = k % nblk
        gw.gw_chi0(probs[b], precision=prec, n_slices=ns, pair_chunk=w.pair_chunk,
                   flags=(0 if b == 0 else acc) | extra)

    for k in range(args.warmup):
        step(k)
    torch.cuda.synchronize()
    _log(t_start, f"{args.warmup} warm-up steps done")
    kern_names = ("mtxel_zy", "mtxel_x", "delta", "chi0_f64", "chi0_tail", "mirror")
    gw.profile_reset()
    gw.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(k)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    gw.profile_enable(False)
    kernels = {k: gw.profile_read(k) for k in kern_names}
    gw.profile_reset()
    _log(t_start, f"{args.steps} timed steps in {elapsed:.3f} s; per-kernel ms/step: " +
         ", ".join(f"{k} {v[1] / args.steps:.2f}" for k, v in kernels.items()))
    # MTXEL alone, after the timed region: one step's 16 x 3,840 pairs as four
    # rows of 4 valence bands (the chunk height of the pipeline) through
    # gw_mtxel with nothing else on the GPU.  In the pipeline MTXEL shares the
    # chip with the contraction, so its event times there include the
    # contraction's share.
    mt_out = torch.empty((4 * nc, ng), dtype=torch.complex128, device=dev)

    def mtxel_step(b):
        for r in range(vbk // 4):
            v0 = b * vbk + 4 * r
            gw.gw_mtxel(w.psi[v0:v0 + 4], psi_c, w.gvec, n, w.volume, out=mt_out)

    mtxel_step(0)
    torch.cuda.synchronize()
    mt_reps = 2
    gw.profile_reset()
    gw.profile_enable(True)
    ev_a, ev_b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev_a.record()
    for k in range(mt_reps):
        mtxel_step(k % nblk)
    ev_b.record()
    torch.cuda.synchronize()
    gw.profile_enable(False)
    mt_alone = ev_a.elapsed_time(ev_b) / mt_reps
    mt_kern = {k: round(gw.profile_read(k)[1] / mt_reps, 3) for k in ("mtxel_zy", "mtxel_x")}
    gw.profile_reset()
    del mt_out
    _log(t_start, f"MTXEL alone: {mt_alone:.2f} ms per step ({mt_kern})")

    pairs_step = vbk * nc
    flops_step = 8.0 * ng * ng * pairs_step * nz
    value = flops_step * args.steps / elapsed / 1e12
    herm = np.real(w.z) == 0.0
    kcs = chunk_pairs(vbk, nc, w.pair_chunk)
    exec_step, alg_step = f64_flops(kcs, ng, herm)
    n_chi, t_chi = kernels["chi0_f64"]
    t_tail = kernels["chi0_tail"][1]
    launches_per_step = max(1, n_chi // max(1, args.steps))
    avg_ms = (t_chi + t_tail) / max(1, n_chi)
    executed = exec_step / launches_per_step / (avg_ms * 1e-3) / 1e12
    algorithmic = alg_step / launches_per_step / (avg_ms * 1e-3) / 1e12
    mt_ms = (kernels["mtxel_zy"][1] + kernels["mtxel_x"][1]) / args.steps
    # MTXEL's algorithmic bytes per step: every band of the step read once and
    # M written once
    mt_bytes = 16.0 * int(np.prod(n)) * (vbk + nc) + 16.0 * pairs_step * ng
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
        "data": "synthetic (seeded Gaussian bands orthonormalised on the grid)",
        "config": {
            "workload": "chi0 precision study at q=0: 72^3 grid, 256x3,840 bands (983,040 "
                        "pairs), 6,031 G, 8 imaginary Gauss-Legendre frequencies, FP64; one "
                        "step = one NV block of 16 valence bands (61,440 pairs, chunks of "
                        "4x1,024) accumulated into chi, 16 steps = the whole chi0",
            "grid": list(n), "pairs": nv * nc, "pairs_per_step": pairs_step, "n_g": ng,
            "n_freq": nz, "pair_chunk": w.pair_chunk, "precision": "fp64",
            "steps_per_build": nblk,
        },
        "pairs_per_s": round(pairs_step * args.steps / elapsed, 1),
        "canonical_flops_per_step": flops_step,
        "kernel_ms_per_step": {k: round(v[1] / args.steps, 3) for k, v in kernels.items()},
        "roofline": {
            "kernel": "chi0_f64_kernel",
            "bound": "mfma",
            "achieved": round(executed, 3),
            "peak": FP64_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": round(executed / FP64_PEAK_TFLOPS, 4),
            "traffic": read_traffic(profile=PROFILE_TRAFFIC_72),
            "flops": "executed: 6 per complex multiply-add on the MFMAs (three real products), "
                     "whole 64x64 tiles on or above the diagonal and 16-pair stages",
            "launches": n_chi,
            "flops_per_launch": exec_step / launches_per_step,
            "avg_launch_ms": round(avg_ms, 4),
            "tail_reduce_ms_per_launch": round(t_tail / max(1, n_chi), 4),
            "algorithmic_tflops": round(algorithmic, 3),
            "algorithmic_flops_per_launch": alg_step / launches_per_step,
        },
        "mtxel": {
            "alone_ms_per_step": round(mt_alone, 3),
            "alone_kernel_ms_per_step": mt_kern,
            "share_of_step": round(mt_alone / (elapsed / args.steps * 1e3), 4),
            "event_ms_per_step_in_pipeline": round(mt_ms, 3),
            "pairs_per_s": round(pairs_step / (mt_alone * 1e-3), 1),
            "algorithmic_bytes_per_step": mt_bytes,
            "achieved_gbs": round(mt_bytes / (mt_alone * 1e-3) / 1e9, 1),
            "hbm_frac": round(mt_bytes / (mt_alone * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "bound": "FP64 MFMA (pruned DFT), not HBM",
        },
    }
    if args.no_legs:
        gw.release()
        print(json.dumps(out), flush=True)
        return

    rows = np.sort(np.random.default_rng(1002).choice(ng, 32, replace=False))
    rows_d = torch.from_numpy(rows).to(dev)

    # whole builds with the autotuner (FP64 tile, split LDS ring), its choices
    # logged to a file; the warm-up step of each build does the tuning
    import tempfile
    tune_fd, tune_path = tempfile.mkstemp(prefix="gw_autotune_", suffix=".txt")
    os.close(tune_fd)
    os.environ["GW_AUTOTUNE_CACHE"] = tune_path

    def build(prec, ns):
        """One whole chi0 (all 16 NV blocks); returns seconds and the 32 rows."""
        step(0, prec, ns, gw.GW_FLAG_AUTOTUNE)  # warm-up (plans, slice buffers, tuning)
        torch.cuda.synchronize()
        gw.profile_reset()
        gw.profile_enable(True)
        t = time.perf_counter()
        for k in range(nblk):
            step(k, prec, ns, gw.GW_FLAG_AUTOTUNE)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        gw.profile_enable(False)
        ks = {k: round(gw.profile_read(k)[1] / nblk, 3)
              for k in ("mtxel_zy", "mtxel_x", "split_prep", "chi0_split", "chi0_split_tail",
                        "chi0_f32", "chi0_f64", "chi0_tail")
              if gw.profile_read(k)[0] > 0}
        gw.profile_reset()
        return dt, chi[:, rows_d].clone(), ks

    flops_build = 8.0 * ng * ng * nv * nc * nz
    t64, ref_rows, ks64 = build("fp64", 0)
    full = {"fp64": {"s_per_build": round(t64, 3), "tflops": round(flops_build / t64 / 1e12, 3),
                     "pairs_per_s": round(nv * nc / t64, 1), "kernel_ms_per_step": ks64}}
    _log(t_start, f"whole FP64 build {t64:.2f} s")
    modes = ([("fp32", 0)] + [("split_bf16", S) for S in args.split_slices] +
             [("split_fp16x9", 4)])
    for prec, ns in modes:
        dt, got, ks = build(prec, ns)
        err = float(torch.linalg.vector_norm(got - ref_rows) / torch.linalg.vector_norm(ref_rows))
        errw = [float(torch.linalg.vector_norm(got[i] - ref_rows[i]) /
                      torch.linalg.vector_norm(ref_rows[i])) for i in range(nz)]
        full[f"{prec}{ns or ''}"] = {
            "precision": prec, "n_slices": ns or None, "s_per_build": round(dt, 3),
            "tflops": round(flops_build / dt / 1e12, 3), "pairs_per_s": round(nv * nc / dt, 1),
            "speedup_vs_fp64": round(t64 / dt, 3), "rel_err_vs_device_fp64_32rows": err,
            "rel_err_per_freq": errw, "kernel_ms_per_step": ks}
        _log(t_start, f"whole {prec} S={ns} build {dt:.2f} s, 32-row error vs device FP64 "
                      f"{err:.2e}")
    out["whole_build"] = full
    del ref_rows
    with open(tune_path) as fh:
        out["whole_build_autotune"] = [ln.strip() for ln in fh if ln.strip()]
    os.environ.pop("GW_AUTOTUNE_CACHE", None)
    os.remove(tune_path)

    # every precision on a 4 x 512-band sample of the same bands against the
    # FP64 oracle (which is also the CPU baseline)
    sv, sc = W2_SAMPLE
    sp = gw.Chi0Problem(n=n, volume=w.volume, psi_v=w.psi[:sv], psi_c=psi_c[:sc],
                        e_v=ev_d[:sv], e_c=ec_d[:sc], gvec=w.gvec, z=w.z)
    dev_rows, dev_full = {}, None
    for prec, ns in [("fp64", 0)] + modes:
        gw.gw_chi0(sp, precision=prec, n_slices=ns, pair_chunk=w.pair_chunk)
        torch.cuda.synchronize()
        dev_rows[f"{prec}{ns or ''}"] = sp.chi[:, rows_d].cpu().numpy()
        if prec == "fp64":
            dev_full = sp.chi.cpu().numpy()
    sp.chi = None
    chi = None
    for pr in probs:
        pr.chi = None
    torch.cuda.empty_cache()
    hv = w.psi[:sv].cpu().numpy()
    hc = psi_c[:sc].cpu().numpy()
    _log(t_start, "device sample results taken; running the oracle on the sample")
    cpu = cpu_baseline_sample(hv, hc, w.e_v[:sv], w.e_c[:sc], w.gvec, w.z, n, w.volume,
                              w.spin, w.pair_chunk, dev_full, dev_rows, rows, nv * nc)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu["baseline"]
    out["oracle_sample"] = cpu["errors"]
    ok = [v for k, v in full.items() if k.startswith("split_bf16") and
          cpu["errors"][k]["rel_err_32rows"] <= 1e-10 and v["rel_err_vs_device_fp64_32rows"] <= 1e-10]
    out["split_bf16_at_1e-10"] = min(ok, key=lambda x: x["n_slices"]) if ok else None
    ok = [v for k, v in full.items() if k.startswith("split_fp16x9") and
          cpu["errors"][k]["rel_err_32rows"] <= 1e-10 and v["rel_err_vs_device_fp64_32rows"] <= 1e-10]
    out["split_fp16x9_at_1e-10"] = min(ok, key=lambda x: x["n_slices"]) if ok else None
    _log(t_start, "done")
    gw.release()
    print(json.dumps(out), flush=True)


def cpu_baseline_sample(hv, hc, e_v, e_c, gvec, z, n, volume, spin, chunk, dev_full, dev_rows,
                        rows, pairs_total):
    """The FP64 oracle on the sample bands (hv x hc), timed on this host; the
    device results of the same sample are compared with it: FP64 in full, every
    precision on the 32 rows."""
    import numpy as np

    import oracle
    info = host_info()
    t0 = time.perf_counter()
    ref = oracle.chi0(hv, hc, e_v, e_c, gvec, z, n, volume, spin=spin, pair_chunk=chunk)
    dt = time.perf_counter() - t0
    pairs = hv.shape[0] * hc.shape[0]
    ng, nz = gvec.shape[0], len(z)
    flops = 8.0 * ng * ng * pairs * nz
    errors = {}
    ref_rows = ref[:, rows]
    for k, got in dev_rows.items():
        errors[k] = {"rel_err_32rows": float(np.linalg.norm(got - ref_rows) /
                                             np.linalg.norm(ref_rows))}
    errors["fp64"]["rel_err_full"] = float(np.linalg.norm(dev_full - ref) / np.linalg.norm(ref))
    errors["sample"] = (f"valence bands 0-{hv.shape[0] - 1} x conduction bands 0-{hc.shape[0] - 1} "
                        f"({pairs} pairs), all {ng} G and {nz} frequencies; rows: 32 G indices "
                        "drawn with numpy default_rng(1002)")
    baseline = {
        "value": round(flops / dt / 1e12, 5),
        "unit": "TFLOP/s",
        "cores": int(info["blas_threads"] or 1),
        "kind": "oracle",
        "sample": f"{pairs} of {pairs_total} pairs (valence 0-{hv.shape[0] - 1} x conduction "
                  f"0-{hc.shape[0] - 1}), all {ng} G and {nz} frequencies; numpy FFT per pair "
                  "(one thread) + BLAS contraction",
        "seconds": round(dt, 2),
        "pairs_per_s": round(pairs / dt, 2),
        "cpu_model": info["cpu_model"],
        "blas": info["blas"],
        "cores_available": info["cores_available"],
        "gpu_rel_err_on_sample": errors["fp64"]["rel_err_full"],
    }
    return {"baseline": baseline, "errors": errors}


def bench_chi0_48cube(args):
    """Workload 1 (48^3 grid, 64 x 960 bands, 2,007 G, 4 real frequencies);
    one step = one gw_chi0 call over all 61,440 pairs."""
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

    # MTXEL alone, after the timed region: the step's 64 x 960 pairs as 16
    # rows of 4 valence bands (the pipeline's chunk rectangle) through
    # gw_mtxel with nothing else on the GPU
    mt_out = torch.empty((4 * p.nc, p.ng), dtype=torch.complex128, device=dev)

    def mtxel_step():
        for v0 in range(0, p.nv, 4):
            gw.gw_mtxel(dp.psi_v[v0:v0 + 4], dp.psi_c, p.gvec, p.n, p.volume, out=mt_out)

    mtxel_step()
    torch.cuda.synchronize()
    mt_reps = 3
    gw.profile_reset()
    gw.profile_enable(True)
    ev_a, ev_b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev_a.record()
    for _ in range(mt_reps):
        mtxel_step()
    ev_b.record()
    torch.cuda.synchronize()
    gw.profile_enable(False)
    mt_alone = ev_a.elapsed_time(ev_b) / mt_reps
    mt_kern = {k: round(gw.profile_read(k)[1] / mt_reps, 3) for k in ("mtxel_zy", "mtxel_x")}
    gw.profile_reset()
    del mt_out
    print(f"[bench] MTXEL alone: {mt_alone:.2f} ms per step ({mt_kern})", file=sys.stderr,
          flush=True)

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
        "mtxel": {
            "alone_ms_per_step": round(mt_alone, 3),
            "alone_kernel_ms_per_step": mt_kern,
            "alone_ms_per_chunk": round(mt_alone / -(-p.nv // 4), 4),
            "pairs_per_chunk": 4 * p.nc,
            "share_of_step": round(mt_alone / (elapsed / args.steps * 1e3), 4),
        },
        "roofline": {
            "kernel": "chi0_f64_kernel",
            "bound": "mfma",
            "achieved": round(executed, 3),
            "peak": FP64_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": round(executed / FP64_PEAK_TFLOPS, 4),
            "traffic": traffic,
            "flops": "executed: 6 per complex multiply-add on the MFMAs (three real products), "
                     "whole 64x64 tiles and 16-pair stages",
            "launches": n_chi,
            "flops_per_launch": exec_per_launch,
            "avg_launch_ms": round(avg_ms, 4),
            "tail_reduce_ms_per_launch": round(t_tail / max(1, n_chi), 4),
            "algorithmic_tflops": round(achieved, 3),
            "algorithmic_flops_per_launch": flops_per_launch,
        },
    }

    # split-BF16 contraction on the same workload: the FP64 chi above is the
    # reference for its error (FP64 parity with the oracle is tested separately)
    ref = gw.gw_chi0(dp, precision="fp64", pair_chunk=chunk).clone()
    splits = []
    for ns in args.split_slices:
        def sstep():  # with the autotuner (the LDS ring); the untimed first call tunes
            gw.gw_chi0(dp, precision="split_bf16", n_slices=ns, pair_chunk=chunk,
                       flags=gw.GW_FLAG_AUTOTUNE)
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
    FP64 and split BF16, with the autotuner (FP64 tile shape, split LDS ring;
    its choices kept in a cache file).  Band sets are drawn on the GPU; every precision is checked against
    the FP64 oracle's direct sums on 16 x 16 sampled entries of the q-points
    with the fewest and the most G."""
    import tempfile

    import numpy as np
    import torch

    import paper_2509_23018_amd as gw
    from workloads import gen

    tune_fd, tune_path = tempfile.mkstemp(prefix="gw_autotune_", suffix=".txt")
    os.close(tune_fd)
    os.environ["GW_AUTOTUNE_CACHE"] = tune_path   # read by the library at its first tuning

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
    osample = keep[:2]                       # q-points checked against the oracle
    srng = np.random.default_rng(1004)
    sidx = {q: (np.sort(srng.choice(int(ngs[q]), 16, replace=False)),
                np.sort(srng.choice(int(ngs[q]), 16, replace=False))) for q in osample}
    dev_entries = {}
    for prec, ns in [("fp64", 0)] + [("split_bf16", k) for k in args.split_slices]:
        flags = gw.GW_FLAG_GRAPH | gw.GW_FLAG_AUTOTUNE

        def call():
            gw.gw_chi0(probs, precision=prec, n_slices=ns, flags=flags)
        t_cap = time.perf_counter()
        call()  # builds plans, captures the graph, runs once
        torch.cuda.synchronize()
        t_cap = time.perf_counter() - t_cap
        gw.profile_reset()
        gw.profile_enable(True)
        dt = _timed(call, max(1, min(args.steps, 3)))
        gw.profile_enable(False)
        gw.profile_reset()
        run = {"precision": prec, "n_slices": ns or None, "s_per_call": round(dt, 4),
               "first_call_s": round(t_cap, 3), "tflops": round(flops / dt / 1e12, 3),
               "pairs_per_s": round(pairs / dt, 1), "autotune": True}
        key = f"{prec}{ns or ''}"
        dev_entries[key] = {}
        for q in osample:
            r_i, c_i = (torch.from_numpy(x).to(dev) for x in sidx[q])
            dev_entries[key][q] = probs[q].chi[:, r_i][:, :, c_i].cpu().numpy()
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
    # the oracle's direct sums on the sampled entries (input preparation:
    # the device bands of those q-points copied to the host)
    import oracle
    t_or = time.perf_counter()
    oerr = {k: {} for k in dev_entries}
    for q in osample:
        pr = probs[q]
        r_i, c_i = sidx[q]
        want = oracle.chi0_entries(pr.psi_v.cpu().numpy(), pr.psi_c.cpu().numpy(),
                                   pr.e_v.cpu().numpy(), pr.e_c.cpu().numpy(),
                                   pr.gvec[r_i], pr.gvec[c_i], z, n, volume)
        for k, got in dev_entries.items():
            oerr[k][int(q)] = float(np.linalg.norm(got[q] - want) / np.linalg.norm(want))
    out["oracle_entries"] = {
        "sample": "16 x 16 entries (rows and columns drawn with numpy default_rng(1004)), all 16 "
                  f"frequencies, q-points {osample} (fewest and most G); oracle direct sums",
        "seconds": round(time.perf_counter() - t_or, 1), "rel_err": oerr}
    with open(tune_path) as fh:
        out["autotune_cache"] = [ln.strip() for ln in fh if ln.strip()]
    os.unlink(tune_path)
    gw.release()
    print(json.dumps(out), flush=True)


ADJOINT_KERNELS = ("mtxel_zy", "mtxel_x", "delta", "bwd_sym", "bwd_gm", "bwd_de", "bwd_de_reduce", "bwd_x",
                   "bwd_yz", "bwd_yz_reduce", "bwd_reduce_c", "bwd_reduce_v")


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
    # the same adjoint reading M kept by the forward (gw_chi0_keep_m, then
    # gw_chi0_backward_from_m): no MTXEL in the adjoint
    m_keep = torch.empty((npairs, ng), dtype=torch.complex128, device=dp.psi_v.device)

    def fwd_keep():
        gw.gw_chi0_keep_m(dp, m_keep, precision="fp64", pair_chunk=chunk)

    def bwd_kept():
        return gw.gw_chi0_backward(dp, w, pair_chunk=chunk, m_keep=m_keep)

    fwd_keep()
    kept_equal = all(torch.equal(a, b) for a, b in
                     zip(bwd_kept(), gw.gw_chi0_backward(dp, w, pair_chunk=chunk)))
    torch.cuda.synchronize()
    t_fwd_keep = _timed(fwd_keep, steps)
    t_bwd_kept = _timed(bwd_kept, steps)
    # The adjoint's GEMMs: g_M = s (conj(Delta) M W + Delta M W^H), two products
    # of 8 flops per (pair, G, G'); where Delta is real (this static workload,
    # and every imaginary or real frequency) one product M (W + W^H).
    nprod = [1 if (complex(zz).real == 0.0 or complex(zz).imag == 0.0) else 2 for zz in p.z]
    gemm_flops = 8.0 * npairs * ng * ng * sum(nprod)
    n_gm, t_gm = kernels["bwd_gm"]
    launches_per_call = max(1, n_gm // steps)
    gm_per_launch = gemm_flops / launches_per_call
    gm_avg_ms = t_gm / max(1, n_gm)
    # executed on the MFMAs: 6 flops per complex multiply-add (three real
    # products), on whole 32 x 64 tiles and 16-wide stages of G
    kc = npairs * nz // launches_per_call
    exec_per_launch = (6.0 * (-(-kc // 32) * 32) * (-(-ng // 64) * 64) * (-(-ng // 16) * 16) *
                       sum(nprod) / nz)
    achieved = exec_per_launch / (gm_avg_ms * 1e-3) / 1e12
    out = {
        "workload": "adjoint_32cube",
        "config": {"grid": list(p.n), "pairs": npairs, "n_g": ng, "n_freq": nz,
                   "pair_chunk": chunk, "precision": "fp64",
                   "grad_chi": "seeded Hermitian N(0,1) matrix (seed 1003)"},
        "data": "synthetic",
        "s_per_forward": round(t_fwd, 5),
        "s_per_adjoint": round(t_bwd, 5),
        "adjoint_over_forward": round(t_bwd / t_fwd, 3),
        "kept_m": {"bytes": npairs * ng * 16, "s_per_forward_keeping_m": round(t_fwd_keep, 5),
                   "s_per_adjoint_from_kept_m": round(t_bwd_kept, 5),
                   "adjoint_over_forward": round(t_bwd_kept / t_fwd, 3),
                   "gradients_equal_to_recomputing_adjoint": kept_equal},
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
            "flops": "executed: 6 per complex multiply-add, whole tiles and stages; one "
                     "product per launch where Delta is real",
            "launches": n_gm,
            "avg_launch_ms": round(gm_avg_ms, 4),
            "flops_per_launch": exec_per_launch,
            "algorithmic_flops_per_launch": gm_per_launch,
            "algorithmic_tflops": round(gm_per_launch / (gm_avg_ms * 1e-3) / 1e12, 3),
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


def _sync_time(fn):
    import torch
    torch.cuda.synchronize()
    t = time.perf_counter()
    r = fn()
    torch.cuda.synchronize()
    return r, time.perf_counter() - t


def _coulomb_q0(gvec):
    """v_G = 4 pi / |G|^2 of the cubic cell at q = 0, the head (G = 0)
    excluded (input preparation)."""
    import numpy as np

    from workloads import gen
    k = np.asarray(gvec, np.float64) * (2.0 * np.pi / gen.CELL_L)
    k2 = (k * k).sum(1)
    return np.where(k2 > 0, 4.0 * np.pi / np.where(k2 > 0, k2, 1.0), 0.0)


def bench_subspace(args):
    """The static subspace (Fast Full-Frequency GW section, Eq. (6)) on the 72^3
    workload's shape and frequencies (256 x 3,840 bands, 6,031 G, 8 imaginary
    frequencies) with shell bands (free-electron-like momentum shells and
    energies): chi0(0) in full plane waves, Diag of the symmetrised
    v^1/2 chi0(0) v^1/2 (q = 0, head excluded), then chi_BB'(z) at 10 % and
    20 % of N_G, against v^1/2 chi v^1/2 of the full plane-wave chi0 at the 8
    frequencies."""
    import numpy as np
    import torch

    import paper_2509_23018_amd as gw
    from workloads import gen

    t_start = time.perf_counter()
    dev = torch.device("cuda", 0)
    w = gen.make_shell_config_device(2, width=1.0, device=dev)
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    ng, nz = w.ng, len(w.z)
    ev_d = torch.from_numpy(w.e_v).to(dev)
    ec_d = torch.from_numpy(w.e_c).to(dev)
    _log(t_start, f"shell bands ready: {w.nv}x{w.nc}, {ng} G")

    def prob(z, chi=None):
        return gw.Chi0Problem(n=w.n, volume=w.volume, psi_v=w.psi_v, psi_c=w.psi_c, e_v=ev_d,
                              e_c=ec_d, gvec=w.gvec, z=z, chi=chi)

    pairs = w.nv * w.nc
    gv = w.gvec.cpu().numpy() if hasattr(w.gvec, "cpu") else np.asarray(w.gvec)
    wt = torch.from_numpy(np.sqrt(_coulomb_q0(gv))).to(dev)
    full, t_full = _sync_time(lambda: gw.gw_chi0(prob(w.z), pair_chunk=w.pair_chunk))
    _log(t_start, f"full plane-wave chi0 at {nz} frequencies: {t_full:.2f} s")
    rows = torch.from_numpy(np.sort(np.random.default_rng(1002).choice(ng, 32, replace=False))).to(dev)
    # the 32 rows of W chi(z) W
    ref_rows = (wt[rows][None, :, None] * full[:, rows] * wt[None, None, :]).contiguous()
    del full
    torch.cuda.empty_cache()
    stat, t_static = _sync_time(lambda: gw.gw_chi0(prob(np.zeros(1, np.complex128)),
                                                  pair_chunk=w.pair_chunk))
    _log(t_start, f"static chi0(0): {t_static:.2f} s")
    chi_s = stat[0].contiguous()
    # the same chi0(0) keeping M of every pair resident in HBM
    # (pairs x N_G complex, 95 GB here), so CHI-Freq skips MTXEL
    (stat_k, m_keep), t_static_keep = _sync_time(
        lambda: gw.gw_chi0_keep_m(prob(np.zeros(1, np.complex128)), pair_chunk=w.pair_chunk))
    keep_equal = bool(torch.equal(stat_k, stat))
    _log(t_start, f"static chi0(0) keeping M ({m_keep.numel() * 16 / 1e9:.1f} GB): "
                  f"{t_static_keep:.2f} s, equal to the plain call: {keep_equal}")
    del stat, stat_k
    runs = []
    for frac in (0.1, 0.2):
        n_eig = int(round(frac * ng))
        (basis, evals, info), t_diag = _sync_time(
            lambda: gw.gw_subspace_basis(chi_s, n_eig, weight=wt, tol=1e-8, seed=7))
        chib, t_sub = _sync_time(lambda: gw.gw_chi0_subspace(prob(w.z), basis, weight=wt,
                                                               pair_chunk=w.pair_chunk))
        chib_m, t_sub_m = _sync_time(lambda: gw.gw_chi0_from_m(prob(w.z), m_keep, basis,
                                                               weight=wt, pair_chunk=w.pair_chunk))
        from_m_equal = bool(torch.equal(chib_m, chib))
        del chib_m
        # W chi(z) W ~ C_s chi_B(z) C_s^H on the 32 rows
        crow = basis[rows].contiguous()
        t1 = gw.gw_zgemm("N", "N", crow[None].expand(nz, -1, -1).contiguous(), chib)
        approx = gw.gw_zgemm("N", "C", t1, basis[None].expand(nz, -1, -1).contiguous())
        err = [float(torch.linalg.vector_norm(approx[i] - ref_rows[i]) /
                     torch.linalg.vector_norm(ref_rows[i])) for i in range(nz)]
        # Diag against the projection of W chi0(0) W on the basis
        wb = (wt[:, None] * basis).contiguous()
        proj = gw.gw_zgemm("C", "N", wb, gw.gw_zgemm("N", "N", chi_s, wb))
        off = float(torch.linalg.vector_norm(proj - torch.diag(evals.to(torch.complex128))) /
                    torch.linalg.vector_norm(evals))
        sub_flops = 8.0 * n_eig * n_eig * pairs * nz
        transf_flops = 8.0 * pairs * ng * n_eig
        runs.append({
            "n_eig": n_eig, "fraction": frac,
            "diag_s": round(t_diag, 3), "diag_info": info,
            "diag_offdiagonal_rel": off,
            "chi_freq_s": round(t_sub, 3),
            "transf_plus_chi_freq_tflops": round((sub_flops + transf_flops) / t_sub / 1e12, 3),
            "subspace_path_s": round(t_static + t_diag + t_sub, 3),
            "speedup_vs_full_plane_waves": round(t_full / (t_static + t_diag + t_sub), 3),
            "chi_freq_from_kept_m_s": round(t_sub_m, 3),
            "chi_freq_from_kept_m_tflops": round(sub_flops / t_sub_m / 1e12, 3),
            "kept_m_equal_to_recomputed": from_m_equal,
            "subspace_path_kept_m_s": round(t_static_keep + t_diag + t_sub_m, 3),
            "speedup_kept_m_vs_full_plane_waves":
                round(t_full / (t_static_keep + t_diag + t_sub_m), 3),
            "rel_err_32rows_per_freq": err,
            "eigenvalue_range": [float(evals[0]), float(evals[-1])],
        })
        _log(t_start, f"n_eig {n_eig}: Diag {t_diag:.2f} s ({info['iterations']} iterations, "
                      f"residual {info['residual']:.1e}), CHI-Freq {t_sub:.2f} s "
                      f"({t_sub_m:.2f} s from kept M, equal: {from_m_equal}), "
                      f"errors {min(err):.2e}..{max(err):.2e}")
        del basis, chib, crow, t1, approx, proj, wb
        torch.cuda.empty_cache()
    out = {"workload": "subspace_72cube",
           "config": {"grid": list(w.n), "pairs": pairs, "n_g": ng, "n_freq": nz,
                      "bands": "shell bands (width 1.0), free-electron energies",
                      "metric": "v^1/2 chi v^1/2, q = 0, head excluded"},
           "data": "synthetic",
           "full_plane_waves_s": round(t_full, 3),
           "full_tflops": round(8.0 * ng * ng * pairs * nz / t_full / 1e12, 3),
           "static_chi0_s": round(t_static, 3),
           "static_chi0_keep_m_s": round(t_static_keep, 3),
           "kept_m_gb": round(m_keep.numel() * 16 / 1e9, 2),
           "kept_m_static_equal": keep_equal,
           "runs": runs}
    del m_keep
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        # the oracle's Diag step (a library Hermitian eigensolver) on the same
        # chi0(0), eigenvalues only, against the device's kept eigenvalues
        import oracle
        wh = wt.cpu().numpy()
        cs = wh[:, None] * chi_s.cpu().numpy() * wh[None, :]
        info = host_info()
        t0 = time.perf_counter()
        lam = np.linalg.eigvalsh(cs)
        dt = time.perf_counter() - t0
        _, want = oracle.static_subspace_basis(np.diag(lam), runs[-1]["n_eig"])
        (bb, ev2, _), _ = _sync_time(lambda: gw.gw_subspace_basis(chi_s, runs[-1]["n_eig"],
                                                                   weight=wt, tol=1e-8, seed=7))
        got = ev2.cpu().numpy()
        out["cpu_baseline"] = {
            "value": round(dt, 2), "unit": "s", "cores": int(info["blas_threads"] or 1),
            "kind": "oracle",
            "sample": f"all eigenvalues of the {ng} x {ng} v^1/2 chi0(0) v^1/2 (numpy eigvalsh)",
            "cpu_model": info["cpu_model"], "blas": info["blas"],
            "gpu_eigenvalue_max_rel_err": float(np.abs(got - want).max() / np.abs(want).max())}
    gw.release()
    print(json.dumps(out), flush=True)


def bench_epsinv(args):
    """The inverse dielectric matrix of Eq. (3) for the 72^3 workload's full
    plane-wave chi0 (6,031 G, 8 imaginary frequencies, seeded recipe bands),
    v_G = 4 pi / |G|^2 with the q = 0 head excluded: block Gauss-Jordan on
    FP64 MFMA GEMMs, 8 N_G^3 flops per frequency."""
    import numpy as np
    import torch

    import paper_2509_23018_amd as gw
    from workloads import gen

    t_start = time.perf_counter()
    dev = torch.device("cuda", 0)
    w = gen.make_config_device(2, device=dev)
    ng, nz = w.ng, len(w.z)
    prob = gw.Chi0Problem(n=w.n, volume=w.volume, psi_v=w.psi_v, psi_c=w.psi_c,
                          e_v=torch.from_numpy(w.e_v).to(dev), e_c=torch.from_numpy(w.e_c).to(dev),
                          gvec=w.gvec, z=w.z)
    chi, t_chi = _sync_time(lambda: gw.gw_chi0(prob, pair_chunk=w.pair_chunk))
    _log(t_start, f"chi0 built in {t_chi:.2f} s")
    del w, prob
    torch.cuda.empty_cache()
    vd = torch.from_numpy(_coulomb_q0(gen.gsphere(gen.CONFIG_SHAPES[2]["r2"]))).to(dev)
    out_t = torch.empty_like(chi)
    gw.gw_epsinv(chi, vd, out=out_t)
    torch.cuda.synchronize()
    steps = max(1, min(args.steps, 5))
    gw.profile_reset()
    gw.profile_enable(True)
    _, dt = _sync_time(lambda: [gw.gw_epsinv(chi, vd, out=out_t) for _ in range(steps)])
    gw.profile_enable(False)
    n_inv, t_inv = gw.profile_read("eps_invert")
    n_zg, t_zg = gw.profile_read("zgemm")
    gw.profile_reset()
    dt /= steps
    flops = 8.0 * ng ** 3 * nz
    # eps eps^-1 = I, on the device
    eps = torch.eye(ng, dtype=torch.complex128, device=dev)[None] - vd[None, :, None] * chi
    prod = gw.gw_zgemm("N", "N", eps, out_t)
    resid = float((prod - torch.eye(ng, dtype=torch.complex128, device=dev)[None]).abs().max())
    del eps, prod
    out = {"workload": "epsinv_72cube",
           "config": {"n_g": ng, "n_freq": nz, "method": "block Gauss-Jordan, 512 columns per step (pivot blocks inverted by 64-column steps)"},
           "data": "synthetic", "chi0_build_s": round(t_chi, 3),
           "s_per_call": round(dt, 4), "tflops": round(flops / dt / 1e12, 3),
           "flops_per_call": flops, "residual_max_abs_eps_epsinv_minus_I": resid,
           "roofline": {"kernel": "block Gauss-Jordan (zgemm updates)", "bound": "mfma",
                        "achieved": round(flops / dt / 1e12, 3), "peak": FP64_PEAK_TFLOPS,
                        "unit": "TFLOP/s", "frac": round(flops / dt / 1e12 / FP64_PEAK_TFLOPS, 4),
                        "traffic": None, "flops": "8 N_G^3 per frequency (algorithmic)",
                        "launches_zgemm": n_zg, "invert_ms_per_call": round(t_inv / max(1, n_inv), 3)}}
    if not args.no_cpu_baseline:
        import oracle
        info = host_info()
        c0 = chi[:1].cpu().numpy()
        t0 = time.perf_counter()
        ref = oracle.epsilon_inverse(c0, vd.cpu().numpy())
        tc = time.perf_counter() - t0
        got = out_t[0].cpu().numpy()
        out["cpu_baseline"] = {
            "value": round(8.0 * ng ** 3 / tc / 1e12, 5), "unit": "TFLOP/s",
            "cores": int(info["blas_threads"] or 1), "kind": "oracle",
            "sample": "frequency 0 of 8 (numpy inverse of the 6,031 x 6,031 eps)",
            "seconds": round(tc, 2), "cpu_model": info["cpu_model"], "blas": info["blas"],
            "gpu_rel_err_on_sample": float(np.linalg.norm(got - ref[0]) / np.linalg.norm(ref[0]))}
    gw.release()
    print(json.dumps(out), flush=True)


GPP_SHAPE = dict(nb=512, ns=128, ng=2007, ne=32)


def bench_gpp(args):
    """The GPP off-diagonal self-energy kernel: Sigma_lm(E) for N_Sigma = 128
    states on 32 energies, 512 bands, 2,007 G (the 48^3 sphere): per (band,
    energy) one GEMM of 128 x 2,007 x 2,007 with the plasmon-pole matrix formed
    inside it and one of 128 x 2,007 x 128.  Flops as the paper counts them
    (Eq. (8), ZGEMM only): 8 (N_Sigma N_G^2 + N_G N_Sigma^2) per (band,
    energy), with the paper's leading factor 2 reported beside it."""
    import numpy as np
    import torch

    import paper_2509_23018_amd as gw
    from workloads import gen

    sh = GPP_SHAPE
    dev = torch.device("cuda", 0)
    inp = gen.gpp_inputs(sh["nb"], sh["ns"], sh["ng"], sh["ne"], seed=1006)
    d = {k: torch.from_numpy(np.ascontiguousarray(inp[k])).to(dev)
         for k in ("m", "omega2", "wtilde", "v")}

    def call():
        return gw.gw_gpp_sigma(d["m"], inp["e_n"], inp["occupied"], inp["energies"], d["omega2"],
                               d["wtilde"], d["v"])

    sig = call()
    torch.cuda.synchronize()
    steps = max(1, min(args.steps, 5))
    gw.profile_reset()
    gw.profile_enable(True)
    _, dt = _sync_time(lambda: [call() for _ in range(steps)])
    gw.profile_enable(False)
    n_t, t_t = gw.profile_read("gpp_t")
    gw.profile_reset()
    dt /= steps
    nb, ns, ng, ne = sh["nb"], sh["ns"], sh["ng"], sh["ne"]
    canon = nb * ne * 8.0 * (ns * ng * ng + ng * ns * ns)
    # gpp_t executes 6 flops per complex multiply-add on whole 64 x 64 tiles and
    # 16-wide stages of G
    tiles = -(-ns // 64) * -(-ng // 64)
    exec_t = 6.0 * tiles * 64 * 64 * (-(-ng // 16) * 16) * ne      # per launch (one band)
    t_avg = t_t / max(1, n_t)
    out = {"workload": "gpp_offdiag", "config": dict(sh), "data": "synthetic",
           "s_per_call": round(dt, 4),
           "tflops": round(canon / dt / 1e12, 3),
           "paper_eq8_tflops": round(2.0 * canon / dt / 1e12, 3),
           "canonical_flops_per_call": canon,
           "roofline": {"kernel": "gpp_t_kernel", "bound": "mfma",
                        "achieved": round(exec_t / (t_avg * 1e-3) / 1e12, 3),
                        "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                        "frac": round(exec_t / (t_avg * 1e-3) / 1e12 / FP64_PEAK_TFLOPS, 4),
                        "traffic": None,
                        "flops": "executed: 6 per complex multiply-add, whole tiles and stages",
                        "launches": n_t, "avg_launch_ms": round(t_avg, 4),
                        "flops_per_launch": exec_t}}
    if not args.no_cpu_baseline:
        import oracle
        info = host_info()
        sb, se = 8, 2
        t0 = time.perf_counter()
        ref = oracle.gpp_sigma_offdiag(inp["m"][:sb], inp["e_n"][:sb], inp["occupied"][:sb],
                                       inp["energies"][:se], inp["omega2"], inp["wtilde"], inp["v"])
        tc = time.perf_counter() - t0
        sub = gw.gw_gpp_sigma(d["m"][:sb].contiguous(), inp["e_n"][:sb], inp["occupied"][:sb],
                              inp["energies"][:se], d["omega2"], d["wtilde"], d["v"]).cpu().numpy()
        cflops = sb * se * 8.0 * (ns * ng * ng + ng * ns * ns)
        out["cpu_baseline"] = {
            "value": round(cflops / tc / 1e12, 5), "unit": "TFLOP/s",
            "cores": int(info["blas_threads"] or 1), "kind": "oracle",
            "sample": f"{sb} of {nb} bands x {se} of {ne} energies",
            "seconds": round(tc, 2), "cpu_model": info["cpu_model"], "blas": info["blas"],
            "gpu_rel_err_on_sample": float(np.linalg.norm(sub - ref) / np.linalg.norm(ref))}
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
