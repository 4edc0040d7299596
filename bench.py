"""Benchmark: Wilson-Dirac even-odd hop bandwidth and CG time-to-solution.

Workload (one GPU): 32^3 x 64 lattice, SU(3) fundamental fermions, links
exp(i 0.3 H) with H Gaussian traceless Hermitian, antiperiodic time,
kappa = 0.13, Gaussian source.  A timed step is one application of the
even-odd hopping block H_{p,1-p} in FP32 (the Dphi kernel that every solve
repeats), alternating the output parity.  value = algorithmic bytes of one
hop (all 4V links once, the input parity field once, the output once) /
mean step time.  The run also reports the FP64 hop, CG time-to-solution at a
1e-10 FP64 true residual (plain FP64 Schur CG and reliable-update mixed
precision), and the FP64 CPU oracle's hop rate on the host cores.

  python bench.py [--steps K] [--warmup W] [--no-cg] [--no-cpu]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def hop_bytes(d, real, sprec, lprec, n_out_sites):
    """Algorithmic bytes of one even-odd hop: 8 links, the input site (read by
    4 neighbours but counted once) and the output site, per output site."""
    bl = {"f64": 8, "f32": 4, "f16s": 2}[lprec]
    bs = {"f64": 8, "f32": 4, "f16s": 2}[sprec]
    link = 8 * (d * d if real else 2 * d * d) * bl
    spin = 2 * (8 * d * bs + (4 if sprec == "f16s" else 0))
    return (link + spin) * n_out_sites


def hop_flops(d, real, n_out_sites):
    return ((64 if real else 128) * d * d + 56 * d) * n_out_sites


def time_hops(ctx, desc, U, A, B, steps, warmup):
    import torch
    nb = ctx.spinor_bytes(desc, 1, 1)
    blocks = [(p, A[(1 - p) * nb:(2 - p) * nb], B[p * nb:(p + 1) * nb]) for p in (0, 1)]

    def step(i):
        p, inp, out = blocks[i & 1]
        ctx.bsm_dslash_eo(desc, U, p, 0, 0.0, None, 1.0, inp, out)

    for i in range(warmup):
        step(i)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for i in range(steps):
        step(i)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps  # ms


def cpu_baseline(lat, Uf, psi, bytes_per_hop, min_seconds=10.0):
    """Oracle even-odd hop on the host cores, doubling the repetition count
    until min_seconds of work (the paper's timing method)."""
    import oracle
    cores = len(os.sched_getaffinity(0))
    oracle.set_num_threads(cores)
    n, total, reps = 1, 0.0, 0
    while total < min_seconds:
        t0 = time.perf_counter()
        for _ in range(n):
            oracle.hop(lat, Uf, psi, parity=reps & 1)
            reps += 1
        total += time.perf_counter() - t0
        n *= 2
    rate = bytes_per_hop * reps / total / 1e9
    return {"value": rate, "unit": "GB/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"{reps} FP64 even-odd hops of the full 32^3x64 SU(3) workload on the host "
                      f"({total:.1f} s, doubling loop); GB/s counts the same algorithmic bytes per hop "
                      f"as the GPU FP32 figure, so the ratio is a ratio of hop rates"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cg", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--dims", type=str, default="64,32,32,32", help="T,LX,LY,LZ")
    ap.add_argument("--only-f32", action="store_true", help="skip the FP64 hop timing")
    ap.add_argument("--copy-calib", type=int, default=0,
                    help="also run N plain 1 GiB device copies (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: multi-GPU runs are not part of this build "
              "(the sharding design is described in DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1401_3733_amd import bsm
    from paper_1401_3733_amd import inputs as gen

    if not os.path.exists(bsm.LIB_PATH):
        from paper_1401_3733_amd import build as _b
        _b.build()
    torch.cuda.set_device(0)
    dims = tuple(int(v) for v in args.dims.split(","))
    lat = gen.Lattice(*dims, bc=(-1, 1, 1, 1))
    kappa = 0.13
    log(f"generating fields {lat} ...")
    t0 = time.time()
    Uf = gen.gauge_links(lat, 3, "near_identity", gen.SEED_GAUGE + 2, eps=0.3)
    psi = gen.gaussian_spinor(lat, 3, gen.SEED_SOURCE + 2)
    log(f"  {time.time() - t0:.1f} s")
    ctx = bsm.Context(lat.dims, lat.bc)
    Uf_dev = bsm.to_device_c128(Uf)
    psi_dev = bsm.to_device_c128(psi)
    res = {}
    Vh = lat.V // 2
    if args.copy_calib:
        src = torch.ones(1 << 30, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(args.copy_calib):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration: {args.copy_calib} copies of 1 GiB")
        del src, dst
    for prec in (("f32",) if args.only_f32 else ("f32", "f64")):
        d = bsm.desc(3, "fund", prec)
        U = ctx.new_gauge(d)
        ctx.bsm_gauge_represent(d, Uf_dev, U)
        A, B = ctx.new_spinor(d), ctx.new_spinor(d)
        ctx.bsm_pack_spinor(d, psi_dev, A)
        steps = args.steps if prec == "f32" else max(10, args.steps // 4)
        log(f"timing {prec} even-odd hop: {steps} steps")
        ms = time_hops(ctx, d, U, A, B, steps, args.warmup)
        nbytes = hop_bytes(3, False, prec, prec, Vh)
        res[prec] = dict(ms=ms, gbs=nbytes / ms / 1e6, tflops=hop_flops(3, False, Vh) / ms / 1e9,
                         bytes=nbytes)
        log(f"  {prec}: {ms * 1e3:.1f} us/hop, {res[prec]['gbs']:.0f} GB/s")
        del U, A, B
    torch.cuda.empty_cache()

    cg = None
    if not args.no_cg:
        cg = {}
        d64 = bsm.desc(3, "fund", "f64")
        U64 = ctx.new_gauge(d64)
        ctx.bsm_gauge_represent(d64, Uf_dev, U64)
        b = ctx.new_spinor(d64)
        ctx.bsm_pack_spinor(d64, psi_dev, b)
        x = ctx.new_spinor(d64)
        for name, prec, lprec, variant in (("plain_f64", "f64", "f64", bsm.SOLVER_PLAIN),
                                           ("mixed_f32", "f32", "f32", bsm.SOLVER_MIXED),
                                           ("mixed_f16s", "f16s", "f32", bsm.SOLVER_MIXED)):
            dl = bsm.desc(3, "fund", prec, lprec)
            Ul = U64 if prec == "f64" else ctx.new_gauge(dl)
            if prec != "f64":
                ctx.bsm_gauge_represent(dl, Uf_dev, Ul)
            prm = bsm.solver_params(kappa, 1e-10, schur=True, variant=variant)
            log(f"CG {name} ...")
            status, st = ctx.bsm_cg_solve(dl, Ul, U64, prm, b, x, check=False)
            cg[name] = dict(status=status, seconds=st["seconds"], iters=st["iters"],
                            true_rel_res=st["true_rel_res"], reliable_updates=st["reliable_updates"],
                            restarts=st["restarts"])
            log(f"  {cg[name]}")
        base = cg["plain_f64"]["seconds"]
        for k in cg:
            cg[k]["speedup_vs_plain_f64"] = base / cg[k]["seconds"] if cg[k]["seconds"] > 0 else None
        del U64, b, x
        torch.cuda.empty_cache()

    cpu = None
    if not args.no_cpu:
        log("CPU oracle baseline ...")
        cpu = cpu_baseline(lat, Uf, psi, res["f32"]["bytes"])
        log(f"  {cpu['value']:.2f} GB/s on {cpu['cores']} threads")

    r32 = res["f32"]
    out = {
        "metric": "Dslash GB/s (% HBM roofline); CG time-to-solution at 1e-10 vs plain FP64",
        "value": round(r32["gbs"], 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r32["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"even-odd Wilson hop, {lat.dims[1]}^3x{lat.dims[0]} SU(3) fundamental, "
                               f"exp(0.3iH) links, antiperiodic time, kappa {kappa}",
                   "lattice": list(lat.dims), "d_R": 3, "rep": "fund", "step": "one FP32 even-odd hop"},
        "roofline": {"bound": "hbm", "achieved": round(r32["gbs"], 1), "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": round(r32["gbs"] / PEAK_HBM_GBS, 4), "traffic": None},
        "tflops_f32": round(r32["tflops"], 2),
        "hop_f64": None if "f64" not in res else {
            "gbs": round(res["f64"]["gbs"], 1), "us": round(res["f64"]["ms"] * 1e3, 2),
            "frac": round(res["f64"]["gbs"] / PEAK_HBM_GBS, 4)},
        "cg": cg,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
