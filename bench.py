"""Benchmark: Wilson-Dirac even-odd hop bandwidth and CG time-to-solution.

Headline workload (one GPU): 32^3 x 64 lattice, SU(3) fundamental fermions,
links exp(i 0.3 H) with H Gaussian traceless Hermitian, antiperiodic time,
kappa = 0.13, Gaussian source.  A timed step is one application of the
even-odd hopping block H_{p,1-p} in FP32 (the Dphi kernel that every solve
repeats), alternating the output parity.  value = algorithmic bytes of one
hop (8 links per output site, the input parity field once, the output once)
/ mean step time, from HIP events on the stream the kernel runs on.

The same run reports time-to-solution at a 1e-10 FP64 true relative residual
against plain FP64 Schur CG on the same GPU for
  * the headline lattice: reliable-update CG with FP32 and FP16+scale inner
    precision;
  * 32^3 x 64 SU(3) two-index symmetric (d_R = 6), kappa 0.125: reliable-
    update CG with FP16+scale spinors (FP32 links, and FP16 links);
  * 24^3 x 48 SU(4) adjoint (d_R = 15), 16 right-hand sides with kappa in
    [0.10, 0.125]: the batched matrix-core solver vs 16 sequential solves;
  * 16^3 x 32 SU(3) fundamental, links exp(i 0.5 H), kappa 0.1335: FGCR with
    the trained parallel-transport network vs plain CG and vs GCR without
    the network (training time reported separately);
the paper's own benchmark (three tasks in its doubling timed loop, rated in
flop/s, for its three theories on the headline lattice), and the FP64 CPU
oracle's hop rate on the host cores.

  python bench.py [--steps K] [--warmup W] [--sections hop,cg,cfg3,cfg4,cfg5,tasks,cpu]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
ALL_SECTIONS = ("hop", "cg", "cfg1", "cfg3", "cfg4", "cfg5", "tasks", "cpu")
# Section III's three theories (N, M): SU(2) stands in for its
# communication-dominated case, whose M = 4 is not one of the supported
# representations of SU(2); SU(3) and SU(6) fundamental are its balanced and
# compute-dominated cases.
TASK_THEORIES = ((2, "fund", "comms"), (3, "fund", "balance"), (6, "fund", "compute"))
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "hop_f32_32x32x32x64_su3_traffic.md")


_T0 = time.time()


def log(msg):
    print(f"[{time.time() - _T0:6.1f} s] {msg}", file=sys.stderr, flush=True)


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


def hop_source_hash():
    """Hash of the sources that define the FP32 hop kernel: counter data taken
    for another version of them is not reported."""
    h = hashlib.sha256()
    for f in ("hop.h", "bsm_internal.h", "spinor_io.h"):
        with open(os.path.join(ROOT, "paper_1401_3733_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per FP32 hop launch from the committed counter summary, or
    None when it is missing or was taken on other kernel sources."""
    if not os.path.exists(TRAFFIC_SUMMARY):
        return None, "no counter summary"
    txt = open(TRAFFIC_SUMMARY).read()
    m = re.search(r"source_hash:\s*(\w+)", txt)
    b = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    if not m or not b:
        return None, "summary without source_hash / hbm_bytes_per_launch"
    if m.group(1) != hop_source_hash():
        return None, "kernel sources changed since the counters were taken"
    return float(b.group(1)), "rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated"


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
    st = torch.cuda.current_stream()   # the stream the library launches on
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for i in range(steps):
        step(i)
    e1.record(st)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps  # ms


def solve_row(status, st, base=None):
    row = dict(status=status, seconds=round(st["seconds"], 4), iters=st["iters"],
               true_rel_res=st["true_rel_res"], reliable_updates=st["reliable_updates"],
               restarts=st["restarts"])
    if base:
        row["speedup_vs_plain_f64"] = round(base / st["seconds"], 3) if st["seconds"] > 0 else None
    return row


def rel_diff(ctx, d64, x, y):
    import torch
    t = torch.empty_like(x)
    ctx.bsm_vec_axpby(d64, 2, 1.0, x, -1.0, y, t)
    return float(np.sqrt(ctx.bsm_vec_dot(d64, 2, t) / ctx.bsm_vec_dot(d64, 2, y)))


# ------------------------------------------------------------- conditioning
def mean_link_and_plaquette(Uf, dims):
    """<Re Tr U>/N over all links and <Re Tr P_munu>/N over all plaquettes
    (mu < nu) of canonical links Uf [V][4][N][N] (lattice axes t, z, y, x;
    direction mu = 0 is t, 1..3 are x, y, z)."""
    T, X, Y, Z = dims
    N = Uf.shape[-1]
    U = Uf.reshape(T, Z, Y, X, 4, N, N)
    axis = {0: 0, 1: 3, 2: 2, 3: 1}
    mean_link = float(np.trace(U, axis1=-2, axis2=-1).real.mean() / N)
    plaq, count = 0.0, 0
    for mu in range(4):
        for nu in range(mu + 1, 4):
            Umu, Unu = U[..., mu, :, :], U[..., nu, :, :]
            Unu_xmu = np.roll(Unu, -1, axis=axis[mu])
            Umu_xnu = np.roll(Umu, -1, axis=axis[nu])
            P = Umu @ Unu_xmu @ np.conj(np.swapaxes(Umu_xnu, -1, -2)) @ np.conj(np.swapaxes(Unu, -1, -2))
            plaq += float(np.trace(P, axis1=-2, axis2=-1).real.sum())
            count += P.size // (N * N)
            del P, Unu_xmu, Umu_xnu
    return mean_link, plaq / count / N


def cg_lanczos(ctx, d64, U64, kappa, b, schur=True, tol=1e-10, max_iter=3000):
    """Extreme eigenvalues of A = M^dag M (M the even-odd Schur operator
    Dhat = 1 - kappa^2 H_eo H_oe on even sites, or D on the full lattice)
    from the coefficients of plain CG on A x = M^dag bhat, run with the
    library's FP64 operator and vector calls: the CG tridiagonal has
    T_kk = 1/alpha_k + beta_(k-1)/alpha_(k-1), T_k,k+1 = sqrt(beta_k)/alpha_k
    (Lanczos connection), and its extreme eigenvalues converge to those of A
    long before CG reaches tol.  cond(M) = sqrt(lambda_max / lambda_min)."""
    import torch
    nb = ctx.spinor_bytes(d64, 1, 1)
    npar = 1 if schur else 2

    def blk(t, p):
        return t[p * nb:(p + 1) * nb]

    if schur:
        tmp = ctx.new_spinor(d64, 1)

        def M(x, y, dag):
            ctx.bsm_dslash_eo(d64, U64, 1, dag, 0.0, None, 1.0, x, tmp)
            ctx.bsm_dslash_eo(d64, U64, 0, dag, 1.0, x, -kappa * kappa, tmp, y)

        bh = ctx.new_spinor(d64, 1)
        ctx.bsm_dslash_eo(d64, U64, 0, 0, 1.0, blk(b, 0), kappa, blk(b, 1), bh)
        new = lambda: ctx.new_spinor(d64, 1)
    else:
        def M(x, y, dag):
            ctx.bsm_dslash_apply(d64, U64, kappa, dag, x, y)

        bh = b
        new = lambda: ctx.new_spinor(d64, 2)
    r, p, t, Ap = new(), new(), new(), new()
    M(bh, r, 1)
    ctx.bsm_vec_axpby(d64, npar, 1.0, r, 0.0, None, p)
    rr = ctx.bsm_vec_dot(d64, npar, r)
    rr0 = rr
    alphas, betas = [], []
    t0 = time.perf_counter()
    while len(alphas) < max_iter and rr > tol * tol * rr0:
        M(p, t, 0)
        M(t, Ap, 1)
        alpha = rr / ctx.bsm_vec_dot(d64, npar, p, Ap)
        ctx.bsm_vec_axpby(d64, npar, 1.0, r, -alpha, Ap, r)
        rr_new = ctx.bsm_vec_dot(d64, npar, r)
        beta = rr_new / rr
        rr = rr_new
        ctx.bsm_vec_axpby(d64, npar, 1.0, r, beta, p, p)
        alphas.append(alpha)
        betas.append(beta)
    torch.cuda.synchronize()
    k = len(alphas)
    diag = np.array([1.0 / alphas[i] + (betas[i - 1] / alphas[i - 1] if i else 0.0) for i in range(k)])
    off = np.array([np.sqrt(betas[i]) / alphas[i] for i in range(k - 1)])
    ev = np.linalg.eigvalsh(np.diag(diag) + np.diag(off, 1) + np.diag(off, -1))
    lo, hi = float(ev[0]), float(ev[-1])
    del r, p, t, Ap
    return {"operator": "Dhat^dag Dhat (even-odd Schur)" if schur else "D^dag D (full lattice)",
            "lambda_min": lo, "lambda_max": hi, "cond_normal": hi / lo, "cond_D": float(np.sqrt(hi / lo)),
            "cg_iters": k, "seconds": round(time.perf_counter() - t0, 3),
            "method": "extreme Ritz values of the CG-Lanczos tridiagonal (FP64 CG to a 1e-10 normal residual); "
                      "lambda_min is an upper estimate of the smallest eigenvalue"}


def conditioning(ctx, d64, U64, kappa, b, Uf_host, dims, schur=True):
    ml, pl = mean_link_and_plaquette(Uf_host, dims)
    out = {"mean_link": ml, "plaquette": pl}
    out.update(cg_lanczos(ctx, d64, U64, kappa, b, schur=schur))
    log(f"  conditioning: {out}")
    return out


def time_block_hops(ctx, d, Ub, A, B, steps):
    """Mean duration of one 16-RHS even-odd block hop (alternating parity),
    HIP events on the stream the library launches on."""
    import torch
    nb = ctx.block_bytes(d) // 2
    ones = np.ones(16)

    def step(i):
        p = i & 1
        ctx.bsm_dslash_eo_block(d, Ub, p, 0, None, None, ones, A[(1 - p) * nb:(2 - p) * nb], B[p * nb:(p + 1) * nb])

    for i in range(4):
        step(i)
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for i in range(steps):
        step(i)
    e1.record(st)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def hop_row(ctx, d, U, A, B, n_out, real, steps, warmup, autotune=True):
    """Autotuned even-odd hop timing with its algorithmic bytes and flops."""
    if autotune:
        ctx.bsm_autotune(d, U)
    ms = time_hops(ctx, d, U, A, B, steps, warmup)
    inv = {0: "f64", 1: "f32", 2: "f16s"}
    nbytes = hop_bytes(d.d_R, real, inv[d.prec], inv[d.link_prec], n_out)
    return {"us": round(ms * 1e3, 2), "gbs": round(nbytes / ms / 1e6, 1),
            "frac": round(nbytes / ms / 1e6 / PEAK_HBM_GBS, 4),
            "tflops": round(hop_flops(d.d_R, real, n_out) / ms / 1e9, 2), "bytes": nbytes,
            "plan": ctx.bsm_get_hop_plan(d)}


# --------------------------------------------------------------- sections
def bench_hop(ctx, lat, Uf_dev, psi_dev, args, bsm):
    import torch
    res = {}
    Vh = lat.V // 2
    for prec in (("f32",) if args.only_f32 else ("f32", "f64")):
        d = bsm.desc(3, "fund", prec)
        U = ctx.new_gauge(d)
        ctx.bsm_gauge_represent(d, Uf_dev, U)
        A, B = ctx.new_spinor(d), ctx.new_spinor(d)
        ctx.bsm_pack_spinor(d, psi_dev, A)
        if not args.no_autotune:
            log(f"autotune {prec} hop ...")
            ctx.bsm_autotune(d, U)
        sweep = {}
        if args.hop_plans and prec == "f32":
            # every listed walk plan in turn (counter runs separate them by
            # dispatch order: warmup + steps dispatches per plan), then the
            # tuned or default plan again
            keep_plan = ctx.bsm_get_hop_plan(d)
            for item in args.hop_plans.split(","):
                order, tc = (int(v) for v in item.split(":"))
                ctx.bsm_set_hop_plan(d, order, tc)
                ms_p = time_hops(ctx, d, U, A, B, args.steps, args.warmup)
                sweep[item] = round(ms_p * 1e3, 2)
                log(f"  plan {item}: {ms_p * 1e3:.1f} us")
            ctx.bsm_set_hop_plan(d, keep_plan["order"], keep_plan["tchunk"])
        plan = ctx.bsm_get_hop_plan(d)
        steps = args.steps if prec == "f32" else max(10, args.steps // 4)
        log(f"timing {prec} even-odd hop: {steps} steps, plan {plan}")
        ms = time_hops(ctx, d, U, A, B, steps, args.warmup)
        nbytes = hop_bytes(3, False, prec, prec, Vh)
        res[prec] = dict(ms=ms, gbs=nbytes / ms / 1e6, tflops=hop_flops(3, False, Vh) / ms / 1e9,
                         bytes=nbytes, plan=plan, steps=steps)
        if sweep:
            res[prec]["plan_sweep_us"] = sweep
        log(f"  {prec}: {ms * 1e3:.1f} us/hop, {res[prec]['gbs']:.0f} GB/s")
        del U, A, B
    torch.cuda.empty_cache()
    return res


def _to_host(ctx, bsm, d64, x, V, d):
    import torch
    c = torch.zeros((V, 4, d), dtype=torch.complex128, device="cuda")
    ctx.bsm_unpack_spinor(d64, x, c)
    h = c.cpu().numpy()
    del c
    return h


class OracleChecks:
    """GPU solutions of full-size workloads, kept on the host for the oracle's
    FP64 true residual ||b - D_W x|| / ||b|| (computed by the oracle's own D_W
    at the end of the run, after the timed GPU sections).  b is the
    generator's source, never read back from the GPU."""

    def __init__(self):
        self.groups = {}

    def group(self, key, lat, Uf_host, rep, workload):
        self.groups[key] = {"lat": lat, "Uf": Uf_host, "rep": rep, "workload": workload, "items": []}

    def add(self, key, label, kappa, b_host, x_host, gpu_res):
        self.groups[key]["items"].append((label, kappa, b_host, x_host, gpu_res))

    def run(self, threads):
        import oracle
        oracle.set_num_threads(threads)
        out = {}
        for key, g in self.groups.items():
            t0 = time.time()
            U = oracle.represent(g["Uf"], g["rep"])
            rows = {}
            for label, kappa, b, x, gpu_res in g["items"]:
                r = oracle.true_residual(g["lat"], U, kappa, b, x)
                rows[label] = {"oracle": r, "gpu": gpu_res}
            del U
            worst = max(v["oracle"] for v in rows.values())
            out[key] = {"workload": g["workload"], "true_rel_res": rows, "max_oracle_true_rel_res": worst,
                        "all_at_or_below_1e-10": bool(worst <= 1e-10),
                        "max_abs_diff_gpu_vs_oracle": max(abs(v["oracle"] - v["gpu"]) for v in rows.values()),
                        "threads": oracle.num_threads(), "seconds": round(time.time() - t0, 1)}
            g["items"] = []
        return out


def bench_cg_cfg2(ctx, lat, Uf_dev, psi_dev, kappa, bsm, Uf_host=None, keep=None):
    """keep (dict or None): receives the host copy of each form's solution
    for the oracle comparison of the CPU leg"""
    import torch
    cg = {}
    d64 = bsm.desc(3, "fund", "f64")
    U64 = ctx.new_gauge(d64)
    ctx.bsm_gauge_represent(d64, Uf_dev, U64)
    b = ctx.new_spinor(d64)
    ctx.bsm_pack_spinor(d64, psi_dev, b)
    x64 = ctx.new_spinor(d64)
    x = ctx.new_spinor(d64)
    x11 = ctx.new_spinor(d64) if keep is not None else None
    base = None
    for name, prec, lprec, variant in (("plain_f64", "f64", "f64", bsm.SOLVER_PLAIN),
                                       ("mixed_f32", "f32", "f32", bsm.SOLVER_MIXED),
                                       ("mixed_f16s", "f16s", "f32", bsm.SOLVER_MIXED),
                                       ("mixed_f16s_f16links", "f16s", "f16s", bsm.SOLVER_MIXED)):
        dl = bsm.desc(3, "fund", prec, lprec)
        Ul = U64 if prec == "f64" else ctx.new_gauge(dl)
        if prec != "f64":
            ctx.bsm_gauge_represent(dl, Uf_dev, Ul)
        prm = bsm.solver_params(kappa, 1e-10, schur=True, variant=variant)
        log(f"CG 32^3x64 SU(3) {name} ...")
        out = x64 if name == "plain_f64" else x
        status, st = warm_solve(lambda: ctx.bsm_cg_solve(dl, Ul, U64, prm, b, out, check=False))
        cg[name] = solve_row(status, st, base)
        if name == "plain_f64":
            base = st["seconds"]
        else:
            cg[name]["x_rel_diff_vs_plain"] = rel_diff(ctx, d64, x, x64)
        if keep is not None:
            keep[name] = _to_host(ctx, bsm, d64, out, lat.V, 3)
            # the error against the oracle is bounded by cond(D) x the true
            # residual: the same solve to 1e-11 shows the bound at work
            prm11 = bsm.solver_params(kappa, 1e-11, schur=True, variant=variant)
            s11, st11 = ctx.bsm_cg_solve(dl, Ul, U64, prm11, b, x11, check=False)
            cg[name]["tol_1e-11"] = dict(status=s11, iters=st11["iters"], true_rel_res=st11["true_rel_res"],
                                         seconds=round(st11["seconds"], 4))
            keep[name + "_tol_1e-11"] = _to_host(ctx, bsm, d64, x11, lat.V, 3)
        log(f"  {cg[name]}")
    if Uf_host is not None:
        log("cfg2 conditioning ...")
        cg["conditioning"] = conditioning(ctx, d64, U64, kappa, b, Uf_host, lat.dims)
    del U64, b, x, x64, x11
    torch.cuda.empty_cache()
    return cg


def bench_cfg1(bsm, gen, keep=None):
    """Plain FP64 CG on the full D^dag D, 4^4 SU(2) fundamental, Haar links,
    kappa 0.12 (latency bound: a correctness and time-to-solution case)."""
    import torch
    c = gen.CONFIGS[1]
    lat = gen.config_lattice(1)
    Uf_host = gen.config_links(1, lat)
    Uf = bsm.to_device_c128(Uf_host)
    ctx = bsm.Context(lat.dims, lat.bc)
    d64 = bsm.desc(2, "fund", "f64")
    U64 = ctx.new_gauge(d64)
    ctx.bsm_gauge_represent(d64, Uf, U64)
    b = ctx.new_spinor(d64)
    ctx.bsm_pack_spinor(d64, bsm.to_device_c128(gen.config_source(1, 2, lat)), b)
    x = ctx.new_spinor(d64)
    log("cfg1 plain FP64 CG on D^dag D ...")
    prm = bsm.solver_params(c["kappa"], 1e-10, schur=False)
    status, st = warm_solve(lambda: ctx.bsm_cg_solve(d64, U64, U64, prm, b, x, check=False))
    out = {"workload": "4^4 SU(2) fund, Haar links, kappa 0.12, CG on the full D^dag D to 1e-10",
           "plain_f64": solve_row(status, st)}
    if keep is not None:
        keep["cfg1"] = _to_host(ctx, bsm, d64, x, lat.V, 2)
    log(f"  {out['plain_f64']}")
    out["conditioning"] = conditioning(ctx, d64, U64, c["kappa"], b, Uf_host, lat.dims, schur=False)
    ctx.close()
    torch.cuda.empty_cache()
    return out


def bench_cfg3(bsm, gen, checks=None):
    """Mixed-precision reliable-update CG, 32^3 x 64 SU(3) two-index symmetric.
    checks (OracleChecks or None): receives every solution for the oracle."""
    import torch
    c = gen.CONFIGS[3]
    lat = gen.config_lattice(3)
    log("cfg3: generating 32^3x64 SU(3) links and source ...")
    Uf_host = gen.config_links(3, lat)
    Uf = bsm.to_device_c128(Uf_host)
    ctx = bsm.Context(lat.dims, lat.bc)
    d64 = bsm.desc(3, "sym", "f64")
    src_host = gen.config_source(3, d64.d_R, lat)
    src = bsm.to_device_c128(src_host)
    if checks is not None:
        checks.group("cfg3", lat, Uf_host, "sym", "32^3x64 SU(3) 2S (d_R=6), every solver form's solution")
    else:
        del src_host
    U64 = ctx.new_gauge(d64)
    ctx.bsm_gauge_represent(d64, Uf, U64)
    b = ctx.new_spinor(d64)
    ctx.bsm_pack_spinor(d64, src, b)
    del src
    x64, x = ctx.new_spinor(d64), ctx.new_spinor(d64)
    out = {"workload": "32^3x64 SU(3) 2S (d_R=6), exp(0.3iH) links, kappa 0.125, Schur CG to 1e-10"}
    base = None
    for name, prec, lprec, variant in (("plain_f64", "f64", "f64", bsm.SOLVER_PLAIN),
                                       ("mixed_f16s", "f16s", "f32", bsm.SOLVER_MIXED),
                                       ("mixed_f16s_f16links", "f16s", "f16s", bsm.SOLVER_MIXED)):
        dl = bsm.desc(3, "sym", prec, lprec)
        Ul = U64 if prec == "f64" else ctx.new_gauge(dl)
        if prec != "f64":
            ctx.bsm_gauge_represent(dl, Uf, Ul)
        prm = bsm.solver_params(c["kappa"], 1e-10, schur=True, variant=variant)
        log(f"cfg3 {name} ...")
        xo = x64 if base is None else x
        status, st = warm_solve(lambda: ctx.bsm_cg_solve(dl, Ul, U64, prm, b, xo, check=False))
        out[name] = solve_row(status, st, base)
        if base is None:
            base = st["seconds"]
        else:
            out[name]["x_rel_diff_vs_plain"] = rel_diff(ctx, d64, x, x64)
        if checks is not None:
            checks.add("cfg3", name, c["kappa"], src_host, _to_host(ctx, bsm, d64, xo, lat.V, 6), st["true_rel_res"])
        log(f"  {out[name]}")
        if prec != "f64":
            del Ul
    x64_keep = x64
    del x
    # the single operator of each precision form, autotuned and timed like the headline hop
    hops = {}
    Vh = lat.V // 2
    for name, prec, lprec in (("f64", "f64", "f64"), ("f32", "f32", "f32"), ("f16s_f32links", "f16s", "f32"),
                              ("f16s_f16links", "f16s", "f16s")):
        dl = bsm.desc(3, "sym", prec, lprec)
        Ul = U64 if prec == "f64" else ctx.new_gauge(dl)
        if prec != "f64":
            ctx.bsm_gauge_represent(dl, Uf, Ul)
        A, B = ctx.new_spinor(dl), ctx.new_spinor(dl)
        canon = torch.zeros((lat.V, 4, 6), dtype=torch.complex128, device="cuda")
        ctx.bsm_unpack_spinor(d64, b, canon)
        ctx.bsm_pack_spinor(dl, canon, A)
        del canon
        log(f"cfg3 hop {name} ...")
        hops[name] = hop_row(ctx, dl, Ul, A, B, Vh, False, 100 if prec != "f64" else 40, 10)
        log(f"  {hops[name]}")
        del A, B
        if prec != "f64":
            del Ul
    out["hop"] = hops
    # fundamental links, the representation formed inside the hop: 8 N x N
    # complex links per output site instead of 8 d x d
    hops_otf = {}
    bl = {"f64": 8, "f32": 4, "f16s": 2}
    for name, prec, lprec in (("f64", "f64", "f64"), ("f32", "f32", "f32"), ("f16s_f32links", "f16s", "f32"),
                              ("f16s_f16links", "f16s", "f16s")):
        dl = bsm.desc(3, "sym", prec, lprec, fundamental_links=True)
        Ul = ctx.new_gauge(dl)
        ctx.bsm_gauge_represent(dl, Uf, Ul)
        A, B = ctx.new_spinor(dl), ctx.new_spinor(dl)
        canon = torch.zeros((lat.V, 4, 6), dtype=torch.complex128, device="cuda")
        ctx.bsm_unpack_spinor(d64, b, canon)
        ctx.bsm_pack_spinor(dl, canon, A)
        del canon
        log(f"cfg3 hop with fundamental links {name} ...")
        ctx.bsm_autotune(dl, Ul)
        ms = time_hops(ctx, dl, Ul, A, B, 100 if prec != "f64" else 40, 10)
        nbytes = (8 * 2 * 9 * bl[lprec] + 2 * (8 * 6 * bl[prec] + (4 if prec == "f16s" else 0))) * Vh
        hops_otf[name] = {"us": round(ms * 1e3, 2), "gbs": round(nbytes / ms / 1e6, 1),
                          "frac": round(nbytes / ms / 1e6 / PEAK_HBM_GBS, 4), "bytes": nbytes,
                          "speedup_vs_stored_links": round(hops[name]["us"] / (ms * 1e3), 3),
                          "plan": ctx.bsm_get_hop_plan(dl)}
        log(f"  {hops_otf[name]}")
        del A, B, Ul
    out["hop_otf"] = hops_otf
    # the solves with fundamental links (FP64 fundamental links for the true
    # residuals and reliable updates too)
    d64o = bsm.desc(3, "sym", "f64", fundamental_links=True)
    U64o = ctx.new_gauge(d64o)
    ctx.bsm_gauge_represent(d64o, Uf, U64o)
    x64o = ctx.new_spinor(d64)
    for name, prec, lprec, variant in (("plain_f64_otf", "f64", "f64", bsm.SOLVER_PLAIN),
                                       ("mixed_f16s_otf", "f16s", "f32", bsm.SOLVER_MIXED),
                                       ("mixed_f16s_f16links_otf", "f16s", "f16s", bsm.SOLVER_MIXED)):
        dl = bsm.desc(3, "sym", prec, lprec, fundamental_links=True)
        Ul = U64o if prec == "f64" else ctx.new_gauge(dl)
        if prec != "f64":
            ctx.bsm_gauge_represent(dl, Uf, Ul)
        prm = bsm.solver_params(c["kappa"], 1e-10, schur=True, variant=variant)
        log(f"cfg3 {name} ...")
        status, st = warm_solve(lambda: ctx.bsm_cg_solve(dl, Ul, U64o, prm, b, x64o, check=False))
        out[name] = solve_row(status, st, base)
        out[name]["x_rel_diff_vs_plain"] = rel_diff(ctx, d64, x64o, x64_keep)
        if checks is not None:
            checks.add("cfg3", name, c["kappa"], src_host, _to_host(ctx, bsm, d64, x64o, lat.V, 6), st["true_rel_res"])
        log(f"  {out[name]}")
        if prec != "f64":
            del Ul
    del U64o, x64o, x64_keep
    log("cfg3 conditioning ...")
    out["conditioning"] = conditioning(ctx, d64, U64, c["kappa"], b, Uf_host, lat.dims)
    ctx.close()
    torch.cuda.empty_cache()
    return out


def bench_cfg4(bsm, gen, checks=None):
    """16 right-hand sides, 24^3 x 48 SU(4) adjoint: batched vs sequential.
    checks (OracleChecks or None): receives the 16 solutions of each of the
    batched (FP32 and F16S inner) and shifted-family solves, and those of
    kappa 0.10, 0.108, 0.117, 0.125 of the sequential FP64 solves, for the
    oracle."""
    import torch
    c = gen.CONFIGS[4]
    lat = gen.config_lattice(4)
    log("cfg4: generating 24^3x48 SU(4) links and 16 sources ...")
    Uf_host = gen.config_links(4, lat)
    Uf = bsm.to_device_c128(Uf_host)
    ctx = bsm.Context(lat.dims, lat.bc)
    d64 = bsm.desc(4, "adj", "f64")
    U = ctx.new_gauge(d64)
    ctx.bsm_gauge_represent(d64, Uf, U)
    del Uf
    kappas = [float(k) for k in c["kappa"]]
    n = len(kappas)
    fb = ctx.spinor_bytes(d64, 2, 1)
    b = ctx.new_spinor(d64, 2, n)
    srcs = []
    for r in range(n):   # one Philox stream per right-hand side
        src = gen.gaussian_spinor(lat, d64.d_R, gen.SEED_SOURCE + 4 + 100 * r)
        ctx.bsm_pack_spinor(d64, bsm.to_device_c128(src), b[r * fb:(r + 1) * fb])
        if checks is not None:
            srcs.append(src)
    sample = (0, 5, 10, 15)
    if checks is not None:
        checks.group("cfg4", lat, Uf_host, "adj", "24^3x48 SU(4) adjoint: all 16 solutions of the batched (FP32 "
                     "and F16S inner) and shifted-family solves; kappa indices 0, 5, 10, 15 of the sequential "
                     "plain FP64 solves")
    torch.cuda.synchronize()
    xb = torch.zeros_like(b)
    xs = torch.zeros_like(b)
    prm = bsm.solver_params(kappas[0], 1e-10, schur=True, max_iter=5000)
    log("cfg4 batched (warm-up call: graph capture, buffers) ...")
    ctx.bsm_batched_solve(d64, U, prm, kappas, b, xb, check=False)
    log("cfg4 batched ...")
    st, stats = ctx.bsm_batched_solve(d64, U, prm, kappas, b, xb, check=False)
    tb = stats[0]["seconds"]
    if checks is not None:
        for r in range(n):
            checks.add("cfg4", f"batched_k{r}", kappas[r], srcs[r],
                       _to_host(ctx, bsm, d64, xb[r * fb:(r + 1) * fb], lat.V, 15), stats[r]["true_rel_res"])
    plan = ctx.bsm_get_block_plan(d64)
    log(f"  {tb:.3f} s, iters {[s['iters'] for s in stats]}, block plan {plan}")
    # the same solve with the F16S inner recurrence (FP16 block fields, links
    # and matrix cores; FP64 reliable updates and true residuals)
    # (replays of 4 iterations, the library's default for F16S)
    dh = bsm.desc(4, "adj", "f16s", "f64")
    xh = torch.zeros_like(b)
    prm_h = bsm.solver_params(kappas[0], 1e-10, schur=True, max_iter=5000, check_every=0)
    log("cfg4 batched F16S (warm-up call) ...")
    ctx.bsm_batched_solve(dh, U, prm_h, kappas, b, xh, check=False)
    log("cfg4 batched F16S ...")
    sth, statsh = ctx.bsm_batched_solve(dh, U, prm_h, kappas, b, xh, check=False)
    tbh = statsh[0]["seconds"]
    if checks is not None:
        for r in range(n):
            checks.add("cfg4", f"batched_f16s_k{r}", kappas[r], srcs[r],
                       _to_host(ctx, bsm, d64, xh[r * fb:(r + 1) * fb], lat.V, 15), statsh[r]["true_rel_res"])
    planh = ctx.bsm_get_block_plan(dh)
    log(f"  {tbh:.3f} s, iters {[s['iters'] for s in statsh]}, block plan {planh}")
    tseq, its, worst, worst_h = 0.0, [], 0.0, 0.0
    log("cfg4 sequential plain FP64 ...")
    # one untimed solve first (the context's plain-CG scratch is allocated there)
    ctx.bsm_cg_solve(d64, U, U, bsm.solver_params(kappas[0], 1e-10, schur=True), b[0:fb], xs[0:fb], check=False)
    for r in range(n):
        p1 = bsm.solver_params(kappas[r], 1e-10, schur=True)
        sl = slice(r * fb, (r + 1) * fb)
        s1, st1 = ctx.bsm_cg_solve(d64, U, U, p1, b[sl], xs[sl], check=False)
        tseq += st1["seconds"]
        its.append(st1["iters"])
        if checks is not None and r in sample:
            checks.add("cfg4", f"sequential_f64_k{r}", kappas[r], srcs[r], _to_host(ctx, bsm, d64, xs[sl], lat.V, 15),
                       st1["true_rel_res"])
        worst = max(worst, rel_diff(ctx, d64, xb[sl], xs[sl]))
        worst_h = max(worst_h, rel_diff(ctx, d64, xh[sl], xs[sl]))
    log(f"  {tseq:.3f} s, iters {its}")
    # the 16-RHS block hop on its own, under the plan the batched solve tuned,
    # on block fields holding the 16 sources
    d32 = bsm.desc(4, "adj", "f32")
    Ub = ctx.new_block_gauge(d32)
    ctx.bsm_gauge_to_block(d32, U, Ub)
    canon = torch.zeros((n, lat.V, 4, 15), dtype=torch.complex128, device="cuda")
    for r in range(n):
        ctx.bsm_unpack_spinor(d64, b[r * fb:(r + 1) * fb], canon[r])
    A, B = ctx.new_block(d32), ctx.new_block(d32)
    ctx.bsm_pack_block(d32, canon, A, n)
    del canon
    torch.cuda.synchronize()
    log("cfg4 block hop timing ...")
    ms = time_block_hops(ctx, d32, Ub, A, B, 40)
    Vh = lat.V // 2
    nbytes = (8 * 15 * 15 * 4 + 16 * 2 * 8 * 15 * 4) * Vh
    flops = 16 * (64 * 15 * 15 + 56 * 15) * Vh
    block_hop = {"us": round(ms * 1e3, 2), "gbs": round(nbytes / ms / 1e6, 1),
                 "frac": round(nbytes / ms / 1e6 / PEAK_HBM_GBS, 4), "tflops": round(flops / ms / 1e9, 2),
                 "bytes": nbytes, "plan": ctx.bsm_get_block_plan(d32),
                 "bytes_model": "8 real FP32 d x d links + 16 x (input + output) FP32 spinors per output site"}
    log(f"  {block_hop}")
    del A, B, Ub
    # the FP16 block hop under the plan the F16S batched solve tuned
    Uh = ctx.new_block_gauge(dh)
    ctx.bsm_gauge_to_block(dh, U, Uh)
    canon = torch.zeros((n, lat.V, 4, 15), dtype=torch.complex128, device="cuda")
    for r in range(n):
        ctx.bsm_unpack_spinor(d64, b[r * fb:(r + 1) * fb], canon[r])
    A, B = ctx.new_block(dh), ctx.new_block(dh)
    ctx.bsm_pack_block(dh, canon, A, n)
    del canon
    torch.cuda.synchronize()
    log("cfg4 FP16 block hop timing ...")
    ms = time_block_hops(ctx, dh, Uh, A, B, 40)
    # links: 8 FP16 d x d (the zero padding of the rows to 16 is not counted);
    # spinors: 16 RHS x 4 d complex FP16 codes + 16 float scales, in and out
    nbytes_h = (8 * 15 * 15 * 2 + 2 * (16 * 4 * 15 * 4 + 16 * 4)) * Vh
    block_hop_h = {"us": round(ms * 1e3, 2), "gbs": round(nbytes_h / ms / 1e6, 1),
                   "frac": round(nbytes_h / ms / 1e6 / PEAK_HBM_GBS, 4), "tflops": round(flops / ms / 1e9, 2),
                   "bytes": nbytes_h, "plan": ctx.bsm_get_block_plan(dh),
                   "speedup_vs_fp32_block_hop": round(block_hop["us"] / (ms * 1e3), 3),
                   "bytes_model": "8 FP16 d x d links (row padding not counted) + 16 x (input + output) FP16 "
                                  "spinors with a float scale per site and RHS, per output site"}
    log(f"  {block_hop_h}")
    del A, B, Uh
    # the shifted family: one source (the first RHS), all 16 kappas in one
    # Krylov space, against 16 sequential plain FP64 solves of that source
    log("cfg4 shifted family (one source, 16 kappas; warm-up call first) ...")
    prm_s = bsm.solver_params(kappas[0], 1e-10, max_iter=5000)
    ctx.bsm_shifted_solve(d64, U, prm_s, kappas, b[0:fb], xb, check=False)
    s_st, s_stats = ctx.bsm_shifted_solve(d64, U, prm_s, kappas, b[0:fb], xb, check=False)
    t_shift = s_stats[0]["seconds"]
    if checks is not None:
        for r in range(n):
            checks.add("cfg4", f"shifted_k{r}", kappas[r], srcs[0],
                       _to_host(ctx, bsm, d64, xb[r * fb:(r + 1) * fb], lat.V, 15), s_stats[r]["true_rel_res"])
        del srcs
    log(f"  {t_shift:.3f} s, iters {[s['iters'] for s in s_stats]}, fell back {[s['fell_back'] for s in s_stats]}")
    tseq1, its1, worst1 = 0.0, [], 0.0
    for r in range(n):
        sl = slice(r * fb, (r + 1) * fb)
        s1, st1 = ctx.bsm_cg_solve(d64, U, U, bsm.solver_params(kappas[r], 1e-10, schur=True), b[0:fb], xs[sl],
                                   check=False)
        tseq1 += st1["seconds"]
        its1.append(st1["iters"])
        worst1 = max(worst1, rel_diff(ctx, d64, xb[sl], xs[sl]))
    log(f"  sequential plain FP64 on the same source: {tseq1:.3f} s")
    shifted = {"workload": "24^3x48 SU(4) adjoint, Haar links, one Gaussian source, kappa linspace(0.10, 0.125, 16)",
               "method": "BiCG with the gamma5 shadow sequence on sigma - H, all kappas as shifts of the largest; "
                         "FP64; members retire at a 0.3e-10 residual estimate, FP64 true residual decides",
               "status": s_st, "seconds": round(t_shift, 4), "iters": [s["iters"] for s in s_stats],
               "fell_back": [s["fell_back"] for s in s_stats],
               "max_true_rel_res": max(s["true_rel_res"] for s in s_stats),
               "sequential_plain_f64": dict(seconds=round(tseq1, 4), iters=its1),
               "speedup_vs_plain_f64": round(tseq1 / t_shift, 3) if t_shift > 0 else None,
               "max_x_rel_diff_vs_plain": worst1}
    cond = {}
    for kk in (kappas[-1], kappas[0]):
        log(f"cfg4 conditioning kappa {kk:.4f} ...")
        cond[f"kappa_{kk:.4f}"] = conditioning(ctx, d64, U, kk, b[0:fb], Uf_host, lat.dims)
    out = {"workload": "24^3x48 SU(4) adjoint (d_R=15, real links), Haar links, 16 RHS, "
                       "kappa linspace(0.10, 0.125, 16), Schur CG to 1e-10 each",
           "kappas": kappas,
           "batched": dict(status=st, seconds=round(tb, 4), iters=[s["iters"] for s in stats], block_plan=plan,
                           max_true_rel_res=max(s["true_rel_res"] for s in stats),
                           reliable_updates=[s["reliable_updates"] for s in stats]),
           "batched_f16s": dict(status=sth, seconds=round(tbh, 4), iters=[s["iters"] for s in statsh],
                                block_plan=planh, max_true_rel_res=max(s["true_rel_res"] for s in statsh),
                                reliable_updates=[s["reliable_updates"] for s in statsh],
                                speedup_vs_plain_f64=round(tseq / tbh, 3) if tbh > 0 else None,
                                max_x_rel_diff_vs_plain=worst_h),
           "sequential_plain_f64": dict(seconds=round(tseq, 4), iters=its),
           "speedup_vs_plain_f64": round(tseq / tb, 3) if tb > 0 else None,
           "max_x_rel_diff_vs_plain": worst,
           "block_hop": block_hop,
           "block_hop_f16": block_hop_h,
           "shifted_family": shifted,
           "conditioning": cond}
    ctx.close()
    torch.cuda.empty_cache()
    return out


def bench_cfg5(bsm, gen, train_steps=300, n_pairs=32, channels=8, large_dims=True):
    """FGCR with the trained PTC network, 16^3 x 32 SU(3), kappa 0.1335."""
    import torch
    c = gen.CONFIGS[5]
    lat = gen.config_lattice(5)
    kappa = c["kappa"]
    log("cfg5: generating 16^3x32 SU(3) links, sources and training solutions ...")
    Uf_host = gen.config_links(5, lat)
    Uf = bsm.to_device_c128(Uf_host)
    ctx = bsm.Context(lat.dims, lat.bc)
    d64 = bsm.desc(3, "fund", "f64")
    d32 = bsm.desc(3, "fund", "f32")
    U64, U32 = ctx.new_gauge(d64), ctx.new_gauge(d32)
    ctx.bsm_gauge_represent(d64, Uf, U64)
    ctx.bsm_gauge_represent(d32, Uf, U32)
    # training solutions x* (Gaussian, own seeds) and the evaluation source
    xs = ctx.new_spinor(d64, 2, n_pairs)
    xs_c = np.stack([gen.gaussian_spinor(lat, 3, gen.SEED_TRAIN + 5 + 1000 * s) for s in range(n_pairs)])
    ctx.bsm_pack_spinor(d64, bsm.to_device_c128(xs_c), xs, n_pairs)
    del xs_c
    b = ctx.new_spinor(d64)
    ctx.bsm_pack_spinor(d64, bsm.to_device_c128(gen.config_source(5, 3, lat)), b)
    f32 = ctx.spinor_bytes(d32, 2, 1)
    r_pairs = torch.zeros(n_pairs * f32 // 4, dtype=torch.float32, device="cuda")
    e_pairs = torch.zeros_like(r_pairs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.bsm_precond_pairs(d64, U64, kappa, n_pairs, xs, [0], r_pairs, e_pairs)
    t_pairs = time.perf_counter() - t0
    W1, W2 = _init_weights(channels, gen.SEED_NET + 5)
    net = torch.cat([torch.from_numpy(W1.astype(np.complex64).ravel()),
                     torch.from_numpy(W2.astype(np.complex64).ravel())]).cuda()
    adam = torch.zeros(4 * net.numel(), dtype=torch.float32, device="cuda")
    log(f"cfg5 training {train_steps} Adam steps on {n_pairs} pairs ...")
    t0 = time.perf_counter()
    losses = ctx.bsm_precond_train(d32, U32, channels, net, adam, r_pairs, e_pairs, n_pairs,
                                   bsm.train_params(lr=5e-3, batch=4, steps=train_steps, seed=gen.SEED_TRAIN + 5))
    t_train = time.perf_counter() - t0
    log(f"  loss {losses[0]:.4f} -> {np.mean(losses[-20:]):.4f} in {t_train:.2f} s")
    x = ctx.new_spinor(d64)
    x0 = ctx.new_spinor(d64)
    rows = {}
    log("cfg5 plain FP64 Schur CG ...")
    s, st = warm_solve(lambda: ctx.bsm_cg_solve(d64, U64, U64, bsm.solver_params(kappa, 1e-10, schur=True), b, x0,
                                                check=False))
    base = st["seconds"]
    rows["plain_f64"] = solve_row(s, st)
    log(f"  {rows['plain_f64']}")
    log("cfg5 mixed FP32 CG ...")
    s, st = warm_solve(lambda: ctx.bsm_cg_solve(
        d32, U32, U64, bsm.solver_params(kappa, 1e-10, schur=True, variant=bsm.SOLVER_MIXED), b, x, check=False))
    rows["mixed_f32"] = solve_row(s, st, base)
    _fgcr_rows(bsm, ctx, d32, d64, U32, U64, kappa, channels, net, b, x, x0, base, rows, "cfg5")
    apply_us = _time_net_apply(bsm, ctx, d32, U32, channels, net, b)
    gain = base - rows["fgcr_net"]["seconds"]
    snap = _cfg5_snapshot_training(bsm, gen, ctx, lat, d32, d64, U32, U64, kappa, channels, b, x, x0, base,
                                   train_steps)
    log("cfg5 conditioning ...")
    cond = conditioning(ctx, d64, U64, kappa, b, Uf_host, lat.dims)
    ctx.close()
    torch.cuda.empty_cache()
    large = bench_cfg5_large(bsm, gen, net, channels, kappa) if large_dims else None
    out = {"workload": "16^3x32 SU(3) fund, exp(0.5iH) links, kappa 0.1335, 1e-10 true residual",
           "net": f"2 PTC layers 1->{channels}->1, 9 paths, FP32",
           "training": dict(pairs=n_pairs, snapshot_iters=[0], steps=train_steps, batch=4, lr=5e-3,
                            seconds=round(t_train, 3), pairs_seconds=round(t_pairs, 3),
                            loss_first=losses[0], loss_last20=float(np.mean(losses[-20:]))),
           "solves": rows,
           "net_apply_us": apply_us,
           "break_even_solves": (round(t_train / gain, 1) if gain > 0 else None),
           "trained_on_cg_snapshots": snap,
           "conditioning": cond,
           "same_net_on_32x32x32x64": large}
    return out


def _val_loss(ctx, d32, U32, channels, net, r_pairs, e_pairs, idx):
    """mean |M(r) - e|^2 / |e|^2 over the pairs idx (library calls)"""
    import torch
    f32 = ctx.spinor_bytes(d32, 2, 1) // 4
    z = torch.zeros(f32, dtype=torch.float32, device="cuda")
    tot = 0.0
    for k in idx:
        r, e = r_pairs[k * f32:(k + 1) * f32], e_pairs[k * f32:(k + 1) * f32]
        ctx.bsm_precond_apply(d32, U32, channels, net, r, z)
        ctx.bsm_vec_axpby(d32, 2, 1.0, z, -1.0, e, z)
        tot += ctx.bsm_vec_dot(d32, 2, z) / ctx.bsm_vec_dot(d32, 2, e)
    return tot / len(idx)


def _cfg5_snapshot_training(bsm, gen, ctx, lat, d32, d64, U32, U64, kappa, channels, b, x, x0, base, train_steps,
                            n_solves=100, snaps=tuple(range(0, 80, 4))):
    """The training set as the workload states it: 2000 residual/error pairs
    from the library's own plain FP64 CG solves (100 solutions x*, 20
    snapshots k = 0, 4, ..., 76 each: e = x* - x_k, r = D e), 1800 for
    training and the last 200 (10 fresh solutions) for validation; the same
    Adam schedule as the 32-pair net; then FGCR(6) with this net."""
    import torch
    n = n_solves * len(snaps)
    f32 = ctx.spinor_bytes(d32, 2, 1)
    log(f"cfg5 snapshot training: {n} pairs from {n_solves} CG solves x {len(snaps)} snapshots ...")
    xs = ctx.new_spinor(d64, 2, n_solves)
    xs_c = np.stack([gen.gaussian_spinor(lat, 3, gen.SEED_TRAIN + 5 + 1000 * (100 + s)) for s in range(n_solves)])
    ctx.bsm_pack_spinor(d64, bsm.to_device_c128(xs_c), xs, n_solves)
    del xs_c
    r_pairs = torch.zeros(n * f32 // 4, dtype=torch.float32, device="cuda")
    e_pairs = torch.zeros_like(r_pairs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.bsm_precond_pairs(d64, U64, kappa, n_solves, xs, list(snaps), r_pairs, e_pairs)
    t_pairs = time.perf_counter() - t0
    del xs
    W1, W2 = _init_weights(channels, gen.SEED_NET + 5)
    net = torch.cat([torch.from_numpy(W1.astype(np.complex64).ravel()),
                     torch.from_numpy(W2.astype(np.complex64).ravel())]).cuda()
    adam = torch.zeros(4 * net.numel(), dtype=torch.float32, device="cuda")
    n_train = n - 200
    t0 = time.perf_counter()
    losses = ctx.bsm_precond_train(d32, U32, channels, net, adam, r_pairs, e_pairs, n_train,
                                   bsm.train_params(lr=5e-3, batch=4, steps=train_steps, seed=gen.SEED_TRAIN + 6))
    t_train = time.perf_counter() - t0
    val = _val_loss(ctx, d32, U32, channels, net, r_pairs, e_pairs, range(n_train, n))
    log(f"  pairs {t_pairs:.2f} s, training {t_train:.2f} s, loss {losses[0]:.4f} -> "
        f"{np.mean(losses[-20:]):.4f}, validation {val:.4f}")
    rows = {}
    prm = bsm.solver_params(kappa, 1e-10, max_iter=20000, restart=6)
    s, st = warm_solve(lambda: ctx.bsm_fgcr_solve(d32, U32, U64, prm, channels, net, b, x, check=False))
    rows["fgcr_net"] = solve_row(s, st, base)
    rows["fgcr_net"].update(fell_back=st["fell_back"], precond_applies=st["precond_applies"],
                            x_rel_diff_vs_plain=rel_diff(ctx, d64, x, x0))
    log(f"  {rows['fgcr_net']}")
    del r_pairs, e_pairs
    torch.cuda.empty_cache()
    return {"pairs": n, "train_pairs": n_train, "validation_pairs": 200, "snapshot_iters": list(snaps),
            "solves": n_solves, "pairs_seconds": round(t_pairs, 3), "training_seconds": round(t_train, 3),
            "steps": train_steps, "loss_first": losses[0], "loss_last20": float(np.mean(losses[-20:])),
            "validation_loss": val, "fgcr": rows}


def bench_cfg5_large(bsm, gen, net, channels, kappa):
    """The network trained on 16^3 x 32 applied, unchanged, on a 32^3 x 64
    lattice of the same link distribution (exp(0.5iH), own seeds): the layers
    are local and gauge covariant, so the weights do not depend on the volume."""
    import torch
    lat = gen.Lattice(64, 32, 32, 32, bc=(-1, 1, 1, 1))
    log("cfg5 transfer: generating 32^3x64 exp(0.5iH) links ...")
    Uf = bsm.to_device_c128(gen.gauge_links(lat, 3, "near_identity", gen.SEED_GAUGE + 105, eps=0.5))
    ctx = bsm.Context(lat.dims, lat.bc)
    d64, d32 = bsm.desc(3, "fund", "f64"), bsm.desc(3, "fund", "f32")
    U64, U32 = ctx.new_gauge(d64), ctx.new_gauge(d32)
    ctx.bsm_gauge_represent(d64, Uf, U64)
    ctx.bsm_gauge_represent(d32, Uf, U32)
    del Uf
    b = ctx.new_spinor(d64)
    ctx.bsm_pack_spinor(d64, bsm.to_device_c128(gen.gaussian_spinor(lat, 3, gen.SEED_SOURCE + 105)), b)
    x, x0 = ctx.new_spinor(d64), ctx.new_spinor(d64)
    rows = {}
    log("cfg5 transfer: plain FP64 Schur CG ...")
    s, st = warm_solve(lambda: ctx.bsm_cg_solve(d64, U64, U64, bsm.solver_params(kappa, 1e-10, schur=True), b, x0,
                                                check=False))
    base = st["seconds"]
    rows["plain_f64"] = solve_row(s, st)
    log(f"  {rows['plain_f64']}")
    s, st = warm_solve(lambda: ctx.bsm_cg_solve(
        d32, U32, U64, bsm.solver_params(kappa, 1e-10, schur=True, variant=bsm.SOLVER_MIXED), b, x, check=False))
    rows["mixed_f32"] = solve_row(s, st, base)
    log(f"  mixed_f32 {rows['mixed_f32']}")
    _fgcr_rows(bsm, ctx, d32, d64, U32, U64, kappa, channels, net, b, x, x0, base, rows, "cfg5 transfer")
    apply_us = _time_net_apply(bsm, ctx, d32, U32, channels, net, b)
    ctx.close()
    torch.cuda.empty_cache()
    return {"workload": "32^3x64 SU(3) fund, exp(0.5iH) links (seed 1105), kappa 0.1335, net trained on 16^3x32",
            "solves": rows, "net_apply_us": apply_us}


def warm_solve(fn):
    """Run a solve twice and keep the second: the first call on a context
    grows its scratch buffers (allocation, zero fill) and is not timed."""
    fn()
    return fn()


def _fgcr_rows(bsm, ctx, d32, d64, U32, U64, kappa, channels, net, b, x, x0, base, rows, tag):
    """GCR(6) without the net, FGCR(6) with the collapsed FP16 net (the
    default) and with the FP32 layers."""
    for name, use_net, layers in (("gcr_no_net", False, 0), ("fgcr_net", True, 0),
                                  ("fgcr_net_layers_f32", True, 1)):
        log(f"{tag} {name} ...")
        prm = bsm.solver_params(kappa, 1e-10, max_iter=20000, restart=6, precond_layers=layers)
        s, st = warm_solve(lambda: ctx.bsm_fgcr_solve(d32, U32, U64, prm, channels, net if use_net else None, b, x,
                                                      check=False))
        rows[name] = solve_row(s, st, base)
        rows[name].update(fell_back=st["fell_back"], precond_applies=st["precond_applies"],
                          x_rel_diff_vs_plain=rel_diff(ctx, d64, x, x0))
        log(f"  {rows[name]}")


def _time_net_apply(bsm, ctx, d32, U32, channels, net, b64, reps=20):
    """Mean duration of one network application, collapsed and layered (HIP
    events on the stream the calls are queued on)."""
    import torch
    f32 = ctx.spinor_bytes(d32, 2, 1)
    r = torch.zeros(f32 // 4, dtype=torch.float32, device="cuda")
    z = torch.zeros_like(r)
    # r: the source rounded to F32 (an internal field with zero padding)
    canon = torch.zeros(int(np.prod(ctx.dims)) * 4 * 3, dtype=torch.complex128, device="cuda")
    ctx.bsm_unpack_spinor(bsm.desc(3, "fund", "f64"), b64, canon)
    ctx.bsm_pack_spinor(d32, canon, r)
    out = {}
    for name, fn in (("collapsed_fp16", ctx.bsm_precond_apply_collapsed), ("layers_f32", ctx.bsm_precond_apply)):
        for _ in range(3):
            fn(d32, U32, channels, net, r, z)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn(d32, U32, channels, net, r, z)
        e1.record()
        e1.synchronize()
        out[name] = round(e0.elapsed_time(e1) * 1e3 / reps, 1)
    log(f"  net apply us {out}")
    return out


def _init_weights(channels, seed):
    """Stay path ~ identity / sqrt(C), hops ~ N(0, 1e-2) complex (Philox)."""
    g = np.random.Generator(np.random.Philox(seed))

    def cg(shape, s):
        z = g.standard_normal(shape + (2,)) * s
        return z[..., 0] + 1j * z[..., 1]

    W1 = cg((channels, 1, 9, 4, 4), 1e-2)
    W2 = cg((1, channels, 9, 4, 4), 1e-2)
    W1[:, 0, 0] += np.eye(4) / np.sqrt(channels)
    W2[0, :, 0] += np.eye(4) / np.sqrt(channels)
    return W1, W2


def measure_copy(bsm, reps=10):
    """Achievable HBM bandwidth of a plain 16-byte copy (bytes read + written
    per launch / mean launch time) and of a read-only sweep, on 1 GiB, each
    the best of a few launch shapes (2048 to 262144 workgroups, ordinary and
    streaming accesses)."""
    import torch
    src = torch.ones(1 << 30, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    part = torch.zeros(262144, dtype=torch.float32, device="cuda")

    def rate(fn, nbytes):
        for _ in range(2):
            fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        e1.synchronize()
        return nbytes * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9

    copy = read = 0.0
    for blocks in (2048, 16384, 65536, 262144):
        for nt in (0, 1):
            copy = max(copy, rate(lambda: bsm.bsm_stream_copy(src, dst, nontemporal=nt, blocks=blocks), 2 << 30))
            read = max(read, rate(lambda: bsm.bsm_stream_read(src, part, blocks=blocks, nontemporal=nt), 1 << 30))
    del src, dst, part
    torch.cuda.empty_cache()
    return copy, read


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
    # one thread: a short sample of the same hop
    oracle.set_num_threads(1)
    t0, reps1 = time.perf_counter(), 0
    while reps1 < 2 or time.perf_counter() - t0 < 2.0:
        oracle.hop(lat, Uf, psi, parity=reps1 & 1)
        reps1 += 1
    rate1 = bytes_per_hop * reps1 / (time.perf_counter() - t0) / 1e9
    oracle.set_num_threads(cores)
    return {"value": rate, "unit": "GB/s", "cores": oracle.num_threads(), "kind": "oracle",
            "value_1_thread": rate1,
            "sample": f"{reps} FP64 even-odd hops of the full 32^3x64 SU(3) workload on the host "
                      f"({total:.1f} s, doubling loop; {reps1} more on one thread); GB/s counts the same "
                      f"algorithmic bytes per hop as the GPU FP32 figure, so the ratio is a ratio of hop rates"}


def _oracle_solve_to(lat, U, kappa, b, x, info, target=1e-13):
    """Continue the oracle's Schur recurrence from the even part of x (a
    solution at a looser tolerance) until the true residual is <= target:
    bhat_e = b_e + kappa H_eo b_o, then x_o = b_o + kappa H_oe x_e."""
    import oracle
    odd = oracle.parity_mask(lat).astype(bool)
    bh = b + kappa * oracle.hop(lat, U, b, parity=0)
    bh[odd] = 0
    xe = x.copy()
    xe[odd] = 0
    res, extra, trig = info["true_res"], 0, target
    while res > target and extra < 4000 and trig > 1e-17:
        xe, it, _ = oracle.cgnr_raw(lat, U, kappa, bh, x0=xe, tol=trig, schur=True)
        extra += it
        x = xe.copy()
        x[odd] = (b + kappa * oracle.hop(lat, U, xe, parity=1))[odd]
        res = oracle.true_residual(lat, U, kappa, b, x)
        trig *= 0.3
    return x, res, extra


def _oracle_reference_job(path, threads):
    """Child process of the CPU leg: the oracle's FP64 Schur CG on the
    headline workload (32^3 x 64 SU(3) fundamental, kappa 0.13) and on the
    two-index one (32^3 x 64 SU(3) 2S, kappa 0.125), each to a 1e-10 true
    residual, timed, then continued to a true residual <= 1e-13 (the
    reference the GPU solutions of that workload are compared with).  Writes
    each solution and a JSON summary next to path (suffixes _2 and _3)."""
    import json as _json
    import oracle
    from paper_1401_3733_amd import inputs as gen
    oracle.set_num_threads(threads)
    for k in (2, 3):
        c = gen.CONFIGS[k]
        lat = gen.config_lattice(k)
        kappa = c["kappa"]
        U = oracle.represent(gen.config_links(k, lat), c["rep"])
        b = gen.config_source(k, oracle.rep_dim(c["N"], c["rep"]), lat)
        t0 = time.perf_counter()
        x, info = oracle.solve(lat, U, kappa, b, tol=1e-10, schur=True)
        t10 = time.perf_counter() - t0
        t1 = time.perf_counter()
        x, res, extra = _oracle_solve_to(lat, U, kappa, b, x, info)
        np.save(f"{path}_{k}.npy", x)
        with open(f"{path}_{k}.json", "w") as f:
            _json.dump({"tts_1e-10_seconds": round(t10, 3), "iters_1e-10": info["iters"],
                        "true_rel_res_1e-10": info["true_res"], "reference_true_rel_res": res,
                        "reference_extra_iters": extra,
                        "reference_extra_seconds": round(time.perf_counter() - t1, 3),
                        "threads": oracle.num_threads()}, f)
        del U, b, x


def start_oracle_reference(threads):
    """Start the oracle's reference solves in a child process (it runs while
    the GPU sections run in this one); returns (process, path)."""
    import multiprocessing as mp
    import tempfile
    path = os.path.join(tempfile.mkdtemp(prefix="bsm_oracle_"), "x_ref")
    proc = mp.get_context("spawn").Process(target=_oracle_reference_job, args=(path, threads), daemon=True)
    proc.start()
    return proc, path


WORKLOAD_NAMES = {2: "32^3x64 SU(3) fund, exp(0.3iH) links, kappa 0.13",
                  3: "32^3x64 SU(3) 2S (d_R=6), exp(0.3iH) links, kappa 0.125"}


def finish_oracle_reference(proc, path, solutions, threads):
    """Wait for the child, then compare each kept GPU solution with the
    oracle's reference solution of its workload.  solutions: {2 or 3:
    {label: host solution}}; returns {2 or 3: summary}."""
    import shutil
    proc.join()
    out = {}
    for k in (2, 3):
        if proc.exitcode != 0 or not os.path.exists(f"{path}_{k}.json"):
            out[k] = {"error": f"oracle reference job failed (exit code {proc.exitcode})"}
            continue
        with open(f"{path}_{k}.json") as f:
            o = json.load(f)
        xr = np.load(f"{path}_{k}.npy")
        nr = np.linalg.norm(xr)
        o["x_rel_err_vs_oracle"] = {lab: float(np.linalg.norm(v - xr) / nr)
                                    for lab, v in solutions.get(k, {}).items()}
        o["workload"] = (f"{WORKLOAD_NAMES[k]}, oracle FP64 Schur CG; timed on {threads} host threads while "
                         "the GPU sections ran in the parent process")
        out[k] = o
        del xr
    shutil.rmtree(os.path.dirname(path), ignore_errors=True)
    return out


def oracle_cfg4_reference(group, threads):
    """The oracle's FP64 Schur CG on the 24^3 x 48 SU(4) adjoint workload for
    the extreme kappas (0.10 with source 0, 0.125 with source 15), each to
    1e-10 (timed) and continued to 1e-13; every kept GPU solution of the same
    (kappa, source) is compared with that reference.  About 4 minutes on 16
    host threads, so only with --oracle-cfg4."""
    import oracle
    oracle.set_num_threads(threads)
    lat = group["lat"]
    U = oracle.represent(group["Uf"], "adj").real.astype(np.complex128)
    items = group["items"]
    kappas = sorted({it[1] for it in items})
    out = {}
    for kappa, r in ((kappas[0], 0), (kappas[-1], 15)):
        # the source of RHS r is the one its batched solution was checked with
        b = next(it[2] for it in items if it[0] == f"batched_k{r}")
        t0 = time.perf_counter()
        x, info = oracle.solve(lat, U, kappa, b, tol=1e-10, schur=True)
        t10 = time.perf_counter() - t0
        t1 = time.perf_counter()
        x, res, extra = _oracle_solve_to(lat, U, kappa, b, x, info)
        nr = np.linalg.norm(x)
        errs = {it[0]: float(np.linalg.norm(it[3] - x) / nr) for it in items
                if it[1] == kappa and it[2] is b}
        out[f"kappa_{kappa:.4f}_source_{r}"] = {
            "tts_1e-10_seconds": round(t10, 3), "iters_1e-10": info["iters"],
            "true_rel_res_1e-10": info["true_res"], "reference_true_rel_res": res,
            "reference_extra_iters": extra, "reference_extra_seconds": round(time.perf_counter() - t1, 3),
            "threads": oracle.num_threads(), "x_rel_err_vs_oracle": errs}
        log(f"  oracle cfg4 kappa {kappa:.4f}: {out[f'kappa_{kappa:.4f}_source_{r}']}")
    return out


def cpu_cfg1(solution):
    """The oracle's FP64 CG on the full D^dag D for the 4^4 SU(2) workload:
    time-to-solution at 1e-10 and the GPU solution against the oracle's
    solution continued to 1e-13."""
    import oracle
    from paper_1401_3733_amd import inputs as gen
    lat = gen.config_lattice(1)
    U = oracle.represent(gen.config_links(1, lat), "fund")
    b = gen.config_source(1, 2, lat)
    k = gen.CONFIGS[1]["kappa"]
    t0 = time.perf_counter()
    _, info = oracle.solve(lat, U, k, b, tol=1e-10, schur=False)
    t = time.perf_counter() - t0
    xr, info13 = oracle.solve(lat, U, k, b, tol=1e-13, schur=False)
    out = {"seconds": round(t, 5), "iters": info["iters"], "true_rel_res": info["true_res"],
           "reference_true_rel_res": info13["true_res"], "cores": oracle.num_threads(),
           "workload": "4^4 SU(2) fund, Haar links, kappa 0.12, oracle FP64 CG on D^dag D to 1e-10"}
    if solution is not None:
        out["x_rel_err_vs_oracle"] = float(np.linalg.norm(solution - xr) / np.linalg.norm(xr))
    return out


def cpu_cg_small():
    """The oracle's FP64 Schur CG to a 1e-10 true residual on the 16^3 x 32
    SU(3) workload (kappa 0.1335, the same links and source as the GPU solves
    of the learned-preconditioner section), on all host cores."""
    import oracle
    from paper_1401_3733_amd import inputs as gen
    lat = gen.config_lattice(5)
    U = oracle.represent(gen.config_links(5, lat), "fund")
    b = gen.config_source(5, 3, lat)
    t0 = time.perf_counter()
    _, info = oracle.solve(lat, U, gen.CONFIGS[5]["kappa"], b, tol=1e-10, schur=True)
    return {"seconds": round(time.perf_counter() - t0, 3), "iters": info["iters"], "true_rel_res": info["true_res"],
            "cores": oracle.num_threads(),
            "workload": "16^3x32 SU(3) fund, exp(0.5iH) links, kappa 0.1335, plain FP64 Schur CG to 1e-10"}


def bench_tasks(bsm, gen, lat, Uf3, min_seconds):
    """The paper's benchmark (Section III): the vector, link x spinor and
    Dphi tasks, each in the library's doubling timed loop (bsm_task_run), for
    the three theories on the headline lattice, FP64 and FP32.  Random
    fields: Haar links for SU(2) and SU(6) (gauge seed 1060 + N), the
    headline exp(0.3iH) links for SU(3); Gaussian sources (seed 2060 + N)."""
    import torch
    rows = []
    for N, rep, role in TASK_THEORIES:
        t0 = time.time()
        Uf = Uf3 if N == 3 else gen.gauge_links(lat, N, "haar", gen.SEED_GAUGE + 60 + N)
        psi = gen.gaussian_spinor(lat, bsm.bsm_rep_dim(N, rep), gen.SEED_SOURCE + 60 + N)
        log(f"tasks SU({N}) {rep}: fields {time.time() - t0:.1f} s")
        ctx = bsm.Context(lat.dims, lat.bc)
        Uf_dev = bsm.to_device_c128(Uf)
        psi_dev = bsm.to_device_c128(psi)
        del Uf, psi
        for prec in ("f64", "f32"):
            d = bsm.desc(N, rep, prec)
            U = ctx.new_gauge(d)
            ctx.bsm_gauge_represent(d, Uf_dev, U)
            inp, out = ctx.new_spinor(d), ctx.new_spinor(d)
            ctx.bsm_pack_spinor(d, psi_dev, inp)
            ctx.bsm_autotune(d, U)          # Dphi runs on the tuned hop plan
            for task in ("vector", "matvec", "dphi"):
                ctx.bsm_task_run(d, task, U, 0.13, inp, out, 0.02)
                it, sec = ctx.bsm_task_run(d, task, U, 0.13, inp, out, min_seconds)
                flops, nbytes = bsm.bsm_task_cost(lat.dims, d, task, lat.bc)
                gbs = nbytes * it / sec / 1e9
                row = dict(theory=f"SU({N}) {rep}", role=role, d_R=d.d_R, prec=prec, task=task,
                           iterations=it, seconds=round(sec, 4), us_per_iter=round(sec / it * 1e6, 2),
                           gflops=round(flops * it / sec / 1e9, 1), gbs=round(gbs, 1),
                           frac_hbm=round(gbs / PEAK_HBM_GBS, 4))
                log(f"  {row}")
                rows.append(row)
            del U, inp, out
        del Uf_dev, psi_dev
        ctx.close()
        torch.cuda.empty_cache()
    return {"lattice": list(lat.dims), "min_seconds": min_seconds,
            "flop_model": "per site: vector 24d; mat-vec 128d^2-8d; Dphi 128d^2+72d",
            "rows": rows}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--sections", type=str, default=",".join(ALL_SECTIONS))
    ap.add_argument("--no-cg", action="store_true", help="skip every solve section")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--dims", type=str, default="64,32,32,32", help="T,LX,LY,LZ of the hop workload")
    ap.add_argument("--only-f32", action="store_true", help="skip the FP64 hop timing")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default hop plan (counter runs: every hop dispatch is the same kernel)")
    ap.add_argument("--task-seconds", type=float, default=0.25,
                    help="minimum timed period of each task of the paper's benchmark")
    ap.add_argument("--hop-plans", type=str, default="",
                    help="also time the FP32 hop under each listed walk plan, 'order:tchunk,...'")
    ap.add_argument("--oracle-cfg4", action="store_true",
                    help="also solve the adjoint workload's extreme kappas with the oracle (about 4 min)")
    ap.add_argument("--copy-calib", type=int, default=0,
                    help="also run N plain 1 GiB device copies (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU (--gpus 1); how the path would shard over several "
              "GPUs is described in the design notes", file=sys.stderr)
        sys.exit(2)
    sections = set(s for s in args.sections.split(",") if s)
    if args.no_cg:
        sections -= {"cg", "cfg1", "cfg3", "cfg4", "cfg5"}
    if args.no_cpu:
        sections.discard("cpu")
    sections.add("hop")

    cores = len(os.sched_getaffinity(0))
    # CPU leg, first part: the oracle's solve of the headline workload runs in
    # a child process on all but two host cores while the GPU sections run
    # (started before this process touches the GPU)
    oracle_job = None
    if "cpu" in sections and "cg" in sections:
        oracle_job = start_oracle_reference(max(1, cores - 2))
        log(f"oracle reference solve of the headline workload started on {max(1, cores - 2)} threads")
    keep = {} if oracle_job is not None else None

    import torch
    from paper_1401_3733_amd import bsm
    from paper_1401_3733_amd import inputs as gen

    bsm.lib()   # raises if the HIP library is not built
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
    if args.copy_calib:
        # a plain copy kernel of known size: its counter readings calibrate
        # the hop's (1 GiB read + 1 GiB written per launch)
        src = torch.ones(1 << 30, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(args.copy_calib):
            bsm.bsm_stream_copy(src, dst)
        torch.cuda.synchronize()
        log(f"calibration: {args.copy_calib} copies of 1 GiB")
        del src, dst
    res = bench_hop(ctx, lat, Uf_dev, psi_dev, args, bsm)
    cg = bench_cg_cfg2(ctx, lat, Uf_dev, psi_dev, kappa, bsm, Uf, keep) if "cg" in sections else None
    del Uf_dev, psi_dev
    ctx.close()
    torch.cuda.empty_cache()
    copy_gbs, read_gbs = measure_copy(bsm)
    log(f"achievable: copy {copy_gbs:.0f} GB/s (1 GiB read + 1 GiB written), read {read_gbs:.0f} GB/s")
    forms = {}
    keep1 = {}
    cfg1 = bench_cfg1(bsm, gen, keep1) if "cfg1" in sections else None
    checks = OracleChecks() if "cpu" in sections else None
    if "cfg3" in sections:
        forms["mixed_precision"] = bench_cfg3(bsm, gen, checks)
    if "cfg4" in sections:
        forms["batched"] = bench_cfg4(bsm, gen, checks)
    if "cfg5" in sections:
        forms["learned_preconditioner"] = bench_cfg5(bsm, gen)
    tasks = bench_tasks(bsm, gen, lat, Uf, args.task_seconds) if "tasks" in sections else None

    cpu = None
    ref = None
    if oracle_job is not None:
        # the rest of the CPU leg times the oracle on every core: wait first
        log("waiting for the oracle reference solves ...")
        sols = {2: keep}
        if checks is not None and "cfg3" in checks.groups:
            sols[3] = {item[0]: item[3] for item in checks.groups["cfg3"]["items"]}
        refs = finish_oracle_reference(*oracle_job, sols, max(1, cores - 2))
        ref = refs[2]
        log(f"  {ref}")
        if "mixed_precision" in forms:
            forms["mixed_precision"]["oracle_reference"] = refs[3]
            log(f"  {refs[3]}")
        keep = sols = None
    if args.oracle_cfg4 and checks is not None and "cfg4" in checks.groups:
        log("oracle FP64 reference solves of the adjoint workload (kappa 0.10 and 0.125) ...")
        forms["batched"]["oracle_reference"] = oracle_cfg4_reference(checks.groups["cfg4"], cores)
    if checks is not None and checks.groups:
        log("oracle FP64 true residuals of the full-size GPU solutions ...")
        for key, v in checks.run(cores).items():
            form = {"cfg3": "mixed_precision", "cfg4": "batched"}[key]
            forms[form]["oracle_check"] = v
            log(f"  {key}: max {v['max_oracle_true_rel_res']:.3e}, |gpu - oracle| <= "
                f"{v['max_abs_diff_gpu_vs_oracle']:.1e}, {v['seconds']} s")
        checks = None
    if "cpu" in sections:
        log("CPU oracle baseline ...")
        cpu = cpu_baseline(lat, Uf, psi, res["f32"]["bytes"])
        log(f"  {cpu['value']:.2f} GB/s on {cpu['cores']} threads, {cpu['value_1_thread']:.2f} GB/s on one")
        log("CPU oracle CG on 16^3x32 ...")
        cpu["cg_tts_16x16x16x32"] = cpu_cg_small()
        log(f"  {cpu['cg_tts_16x16x16x32']}")
        log("CPU oracle CG on 4^4 ...")
        cpu["cg_tts_4x4x4x4"] = cpu_cfg1(keep1.get("cfg1"))
        log(f"  {cpu['cg_tts_4x4x4x4']}")
        if ref is not None:
            cpu["cg_32x32x32x64"] = ref

    r32 = res["f32"]
    traffic, traffic_note = measured_traffic()
    out = {
        "metric": "Dslash GB/s (% HBM roofline); CG time-to-solution at 1e-10 vs plain FP64",
        "value": round(r32["gbs"], 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": r32["steps"],
        "warmup": args.warmup,
        "ms_per_step": r32["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"even-odd Wilson hop, {lat.dims[1]}x{lat.dims[2]}x{lat.dims[3]}x{lat.dims[0]} "
                               f"SU(3) fundamental, exp(0.3iH) links, antiperiodic time, kappa {kappa}",
                   "lattice": list(lat.dims), "d_R": 3, "rep": "fund", "step": "one FP32 even-odd hop",
                   "hop_plan": r32["plan"]},
        "roofline": {"bound": "hbm", "achieved": round(r32["gbs"], 1), "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": round(r32["gbs"] / PEAK_HBM_GBS, 4), "traffic": traffic,
                     "algorithmic_bytes_per_launch": r32["bytes"], "traffic_source": traffic_note,
                     "achievable_gbs": {"copy": round(copy_gbs, 1), "read": round(read_gbs, 1)}},
        "tflops_f32": round(r32["tflops"], 2),
        **({"hop_plan_sweep_us": r32["plan_sweep_us"]} if "plan_sweep_us" in r32 else {}),
        "hop_f64": None if "f64" not in res else {
            "gbs": round(res["f64"]["gbs"], 1), "us": round(res["f64"]["ms"] * 1e3, 2),
            "frac": round(res["f64"]["gbs"] / PEAK_HBM_GBS, 4), "plan": res["f64"]["plan"]},
        "cg": cg,
        "cfg1": cfg1,
        "forms": forms or None,
        "paper_tasks": tasks,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
