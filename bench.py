#!/usr/bin/env python3
"""Benchmark of the Poisson-lognormal MAP hot path on one MI355X.

Workload (the 256^3 selection workload): 256^3 periodic grid, 500 Mpc/h box,
Gaussian log-field with P(k) = A k^-1.5 exp(-(2k)^2), sigma_G = 1.5, radial
selection w = exp(-(r/200)^2) with 20% of 8^3 blocks masked, nbar = 0.5,
unit bias; synthetic inputs from a fixed seed, resident in HBM before timing.

A step is one full inexact Newton-Krylov MAP solve from s0 = mu to
||g|| / ||g0|| < 1e-6 in FP64: gradients, Hessian-vector products, Krylov
dots and updates, line searches.  `value` is the number of Hessian-vector
products performed in the timed steps divided by their wall time.

Also reported (not part of `value`):
  roofline      -- the in-solver spectral HVP (5 passes) timed in isolation
                   with HIP events on the plan's stream (median of 200
                   calls after 20 warm-up calls), against 8 TB/s
  mixed         -- the same solve with FP32 FFTs/HVPs and FP64 reductions
  adjoint       -- adjoint solve of L = sum (s* - s_true)^2 at the MAP
  nlcg          -- the paper-literal Krylov step (eq. New5 step length,
                   nonlinear-CG search vectors), FP64, same tolerance
  linear_bias   -- the MAP with a non-local linear bias (a smoothing b_hat),
                   lognormal and Gaussian priors: solve time and the
                   real-space HVP with its byte model
  estimators    -- the paper's comparison estimators (Gaussian-prior MAP,
                   LSQ-Wiener filter, inverse weighting, lognormal prior
                   construction) with the correlation coefficient and
                   Euclidean distance of each reconstruction, MAP included,
                   against the true overdensity
  batched       -- 64 independent reconstructions, n in {32, 48, 64, 96},
                   solved together (mixed precision) vs one after another
                   (plain FP64)
  cpu_baseline  -- the CPU oracle's spectral HVP on the host cores

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0
# FFT tile schedules chosen by pl_plan_autotune on MI355X for the benchmark
# grids (the autotuner reads them instead of timing when the key is present)
TUNE_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_0911_1407_amd",
                          "tune_cache_gfx950.txt")


# Memory-side traffic of one FP64 spectral HVP on the 256^3 selection
# workload: FETCH_SIZE and WRITE_SIZE (rocprofv3 --pmc) of the five passes,
# each scaled by what the counter reads for a 1 GiB device copy in the same
# program.  It holds for the kernel sources it was measured on (sha256 of
# paper_0911_1407_amd/csrc/*.hip and *.hpp, sorted by path, first 16 hex
# digits) and the FP64 schedule it ran; otherwise the bench reports null.
MEASURED_TRAFFIC = {
    "sel256": {"src_sha": "2e23c239b2167119", "fp64_schedule": [5, 0, 0, 0, 2, 2, 30],
               "bytes_per_hvp": 1685961696},
}


def kernel_sources_sha():
    import glob
    import hashlib
    csrc = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_0911_1407_amd", "csrc")
    paths = sorted(glob.glob(os.path.join(csrc, "*.hip")) + glob.glob(os.path.join(csrc, "*.hpp")))
    h = hashlib.sha256()
    for path in paths:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(workload, fp64_schedule):
    m = MEASURED_TRAFFIC.get(workload)
    if m is None or m["src_sha"] != kernel_sources_sha() or list(m["fp64_schedule"]) != list(fp64_schedule):
        return None
    return m["bytes_per_hvp"]


def hvp_bytes(n, p, spectral=True):
    """Algorithmic HBM bytes of one Hessian-vector product.

    Spectral (in-solver) form: 5 passes; passes 1-4 read and write the
    half spectrum (2 * 2p * Nh each), the z pass also reads d (p N, 8 bytes
    in FP64, 4 in FP32), pass 5 reads the transformed field and p_hat and
    writes H p_hat (3 * 2p * Nh).  Total p N + 22 p Nh.
    """
    N = n[0] * n[1] * n[2]
    Nh = n[0] * n[1] * (n[2] // 2 + 1)
    if spectral:
        return p * N + 22 * p * Nh
    return 4 * p * N + 16 * p * Nh


def linear_bias_hvp_bytes(n, lognormal):
    """Algorithmic FP64 bytes of one real-space linear-bias HVP with a cached
    linearisation (pl_linear_bias_hessvec, x = NULL): v to half spectrum (3
    passes), the spectral HVP, back to real space (3).  Lognormal prior: x^-1,
    y^-1, z (keeps q, times phi', sums phi'' B u q^2), y, x(b_hat), y^-1,
    z (times N/y^2), y, x(b_hat), y^-1, z (phi' g + phi'' B u q), y, x + prior.  Gaussian prior:
    x^-1, x(b_hat), y^-1, z (times N/y^2), y, x(b_hat), x + prior."""
    N = n[0] * n[1] * n[2]
    Nh = n[0] * n[1] * (n[2] // 2 + 1)
    fwd = (8 * N + 16 * Nh) + 32 * Nh + 32 * Nh          # z r2c, y, x
    inv = 32 * Nh + 32 * Nh + (16 * Nh + 8 * N)          # x, y, z c2r
    col, xmul, xadd = 32 * Nh, 40 * Nh, 48 * Nh          # plain, x(b_hat) (+ table), x + prior
    zhvp = 32 * Nh + 8 * N                               # z pass with a diagonal
    if lognormal:
        hvp = 7 * col + 2 * xmul + xadd + (32 * Nh + 24 * N) + zhvp + (32 * Nh + 24 * N)
    else:
        hvp = col + 2 * xmul + col + zhvp + col + xadd
    return fwd + hvp + inv


def cg_step_bytes(n, p):
    """Algorithmic bytes of one fused CG step (five passes with the Krylov
    updates): p N + 32 p Nh."""
    N = n[0] * n[1] * n[2]
    Nh = n[0] * n[1] * (n[2] // 2 + 1)
    return p * N + 32 * p * Nh


def batched_workload(dev, rtol):
    """64 independent reconstructions (n in {32, 48, 64, 96}) solved together,
    in mixed precision and in plain FP64, against sequential single-grid
    solves of the same instances in the same two precisions (so that the
    gain of batching and the gain of precision are reported apart)."""
    import torch
    from paper_0911_1407_amd import synth
    from paper_0911_1407_amd.binding import Batch, Plan, make_opts, pl_newton_krylov_solve
    t0 = time.time()
    insts = synth.batch_instances(count=64)
    print(f"# generated 64 batch instances in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    bt = Batch(insts, precision="mixed", device=dev)
    bt.autotune(TUNE_CACHE)

    def run_batch(prec):
        bt.solve(rtol=rtol, precision=prec)  # warm-up (also builds the CG graph)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s_list, infos = bt.solve(rtol=rtol, precision=prec)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, infos, s_list

    def run_sequential(prec):
        t = 0.0
        infos = []
        for it in insts:
            pp = Plan(it["n"], it["box"], precision="mixed", device=dev)
            pp.set_instance(it)
            s0 = torch.full(it["n"], float(it["mu"]), dtype=torch.float64, device=dev)
            pl_newton_krylov_solve(pp.h, s0, make_opts(rtol=rtol, precision=prec))  # warm-up
            s0.fill_(float(it["mu"]))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            infos.append(pl_newton_krylov_solve(pp.h, s0, make_opts(rtol=rtol, precision=prec)).as_dict())
            torch.cuda.synchronize()
            t += time.perf_counter() - t0
            pp.close()
        return t, infos

    out = {"instances": len(insts)}
    for name, prec, p in (("mixed", 1, 4), ("fp64", 0, 8)):
        tb, binfos, s_list = run_batch(prec)
        parity = batch_oracle_parity(insts, s_list)
        ts, sinfos = run_sequential(prec)
        nconv = sum(1 for i in binfos if i["status"] == 0)
        # algorithmic bytes of the CG steps each instance took, over the
        # whole batched solve's wall time: a lower bound on the bandwidth
        # of the batched passes (gradients, line searches and launch gaps
        # are in the time, not in the bytes)
        cg_bytes = sum(i["cg_its"] * cg_step_bytes(it["n"], p) for i, it in zip(binfos, insts))
        out[name] = {"ms_batched": 1e3 * tb, "ms_sequential": 1e3 * ts, "speedup_batching": ts / tb,
                     "instances_per_s_batched": len(insts) / tb, "instances_per_s_sequential": len(insts) / ts,
                     "converged": nconv, "cg_its_total": sum(i["cg_its"] for i in binfos),
                     "fp64_steps": sum(i["fp64_steps"] for i in binfos),
                     "cg_algorithmic_bytes": cg_bytes, "cg_bytes_per_s_lower_bound_GBs": cg_bytes / tb / 1e9,
                     "oracle_parity": parity}
        print(f"# batch {name}: {1e3 * tb:.0f} ms batched vs {1e3 * ts:.0f} ms sequential "
              f"({ts / tb:.2f}x, {nconv}/64 converged, CG bytes {cg_bytes / tb / 1e9:.0f} GB/s over the solve; "
              f"max rel-L2 vs the stored oracle MAPs {parity['max_rel_l2'] if parity else None})",
              file=sys.stderr, flush=True)
    out["speedup_mixed_batched_vs_fp64_sequential"] = out["fp64"]["ms_sequential"] / out["mixed"]["ms_batched"]
    return out


def oracle_parity(workload, inst, fields):
    """Relative L2 error of GPU MAP fields against the stored oracle MAP
    (tests/golden/<workload>_map.json, written by the oracle alone) over its
    sampled cells, and the worst cell in units of max(|ref|, 1e-2 max|ref|);
    None when no stored result exists or the inputs differ from the stored
    run's."""
    import hashlib
    if workload is None:
        return None
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests", "golden", f"{workload}_map.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        ref = json.load(f)
    sha = hashlib.sha256(np.ascontiguousarray(inst["counts"]).tobytes()).hexdigest()
    if sha != ref["inputs"]["counts_sha256"]:
        return None
    cells = np.asarray(ref["cells"])
    r = np.asarray(ref["s_star_cells"])
    scale = np.maximum(np.abs(r), 1e-2 * np.abs(r).max())
    out = {"sample_cells": int(cells.size), "oracle_rtol": ref["oracle_solve"]["rtol"]}
    for name, t in fields.items():
        a = t.detach().cpu().numpy().ravel()[cells]
        out[name] = {"rel_l2": float(np.linalg.norm(a - r) / np.linalg.norm(r)),
                     "max_cell_rel": float(np.max(np.abs(a - r) / scale))}
    return out


def batch_oracle_parity(insts, s_list):
    """Each batched MAP against the stored oracle MAP of its instance
    (tests/golden/batch64_map.json) over that instance's sampled cells: the
    largest relative L2 error and the largest worst-cell error (units of
    max(|ref|, 1e-2 max|ref|)) over the instances; None when no stored result
    exists or an instance's inputs differ from the stored run's."""
    import hashlib
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests", "golden", "batch64_map.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        ref = json.load(f)["instances"]
    if len(ref) != len(insts):
        return None
    rel, worst = 0.0, 0.0
    for it, s, rec in zip(insts, s_list, ref):
        if hashlib.sha256(np.ascontiguousarray(it["counts"]).tobytes()).hexdigest() != rec["inputs"]["counts_sha256"]:
            return None
        cells = np.asarray(rec["cells"])
        r = np.asarray(rec["s_star_cells"])
        a = s.detach().cpu().numpy().ravel()[cells]
        rel = max(rel, float(np.linalg.norm(a - r) / np.linalg.norm(r)))
        worst = max(worst, float(np.max(np.abs(a - r) / np.maximum(np.abs(r), 1e-2 * np.abs(r).max()))))
    return {"instances": len(insts), "oracle_rtol": ref[0]["oracle_solve"]["rtol"], "max_rel_l2": rel,
            "max_cell_rel": worst}


def cpu_oracle_baseline(inst, v, full=False):
    """The CPU oracle (plain FP64 numpy / scipy.fft on the host cores) timed
    on bounded samples of the benchmark's workloads.  value: oracle spectral
    HVPs per second at the workload's size (up to 40 HVPs, about 15 s).
    time_to_map: the oracle's inexact Newton-Krylov solve of the 32^3 plain
    workload (rtol 1e-8) and sequential solves of the first 8 instances of
    the 64-instance batched workload (rtol 1e-6), with Newton / CG counts;
    with full=True (--cpu-full) also the 256^3 selection workload's solve
    and adjoint (rtol 1e-6) and all 64 batch instances, which take minutes
    (the 256^3 bias workload's oracle MAP takes hours; its time at rtol
    1e-10 is recorded by tests/golden/make_golden.py)."""
    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    from oracle import adjoint as o_adj
    from oracle import dft as o_dft
    from oracle.grid import Problem
    from oracle.model import hess_diag
    from oracle.newton import SpectralOps, newton_krylov
    from paper_0911_1407_amd import synth

    def problem(it):
        return Problem(it["n"], it["box"], it["w"], it["counts"], it["pk"], it["amp"], it["mu"], it["nbar"],
                       it["beta"], 0.0)

    def timed_solve(it, rtol, precond="mean", name=None):
        # progress lines (one per Newton step) only for the long full-size
        # solves; printing is outside the oracle's arithmetic
        prog = None
        if name:
            def prog(k, rg, cg):
                print(f"# cpu oracle {name}: newton {k} rel_grad {rg:.2e} cg {cg}", file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        s_, info = newton_krylov(problem(it), rtol=rtol, max_newton=200, max_cg=5000, precond=precond,
                                 progress=prog)
        return s_, {"s": time.perf_counter() - t0, "newton_its": int(info["newton_its"]),
                    "cg_its": int(info["cg_its"]), "status": info["status"], "rtol": rtol, "precond": precond}

    P = problem(inst)
    ops = SpectralOps(P)
    d = hess_diag(P, inst["s_true"])
    vh = np.fft.rfftn(v)
    ops.hessvec(d, vh)
    reps = 0
    t0 = time.perf_counter()
    while True:
        ops.hessvec(d, vh)
        reps += 1
        if time.perf_counter() - t0 > 15.0 or reps >= 40:
            break
    t_hvp = (time.perf_counter() - t0) / reps
    ttm = {}
    _, ttm["plain32"] = timed_solve(synth.config_instance("plain32"), 1e-8)
    insts = synth.batch_instances(count=64)
    subset = insts if full else insts[:8]
    recs = []
    for k, it in enumerate(subset):
        recs.append(timed_solve(it, 1e-6)[1])
        if full:
            print(f"# cpu oracle batch instance {k + 1}/{len(subset)} n={it['n'][0]}: {recs[-1]['s']:.1f} s",
                  file=sys.stderr, flush=True)
    ttm["batch64_sequential"] = {"instances": len(subset), "n": [int(it["n"][0]) for it in subset],
                                 "s": sum(r["s"] for r in recs), "cg_its": sum(r["cg_its"] for r in recs),
                                 "rtol": 1e-6}
    if full:
        sel = synth.config_instance("sel256")
        s_sel, ttm["sel256"] = timed_solve(sel, 1e-6, name="sel256")
        print(f"# cpu oracle sel256 solve: {ttm['sel256']}", file=sys.stderr, flush=True)
        # the adjoint of L = sum (s* - s_true)^2 at that MAP
        _, dL = o_adj.squared_error_loss(s_sel, sel["s_true"])
        t0 = time.perf_counter()

        def aprog(k, rn):
            print(f"# cpu oracle sel256 adjoint: cg {k} residual {rn:.3e}", file=sys.stderr, flush=True)

        _, its = o_adj.adjoint_pcg(problem(sel), s_sel, dL, rtol=1e-6, max_cg=50000, progress=aprog)
        ttm["sel256_adjoint"] = {"s": time.perf_counter() - t0, "cg_its": int(its), "rtol": 1e-6}
        print(f"# cpu oracle sel256 adjoint: {ttm['sel256_adjoint']}", file=sys.stderr, flush=True)
    cpu_model = None
    try:
        with open("/proc/cpuinfo") as f:
            cpu_model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), None)
    except OSError:
        pass
    n = inst["n"]
    return {"value": 1.0 / t_hvp, "unit": "HVP/s", "cores": o_dft._WORKERS, "kind": "oracle",
            "cpu_model": cpu_model,
            "sample": f"{reps} oracle spectral HVPs (scipy rfftn/irfftn on {o_dft._WORKERS} threads, FP64) on "
                      f"the same {n[0]}^3 data at s = s_true, elementwise numpy single-threaded; time_to_map: "
                      f"oracle Newton-Krylov solves (plain32 at rtol 1e-8, {len(subset)} batch instances at "
                      f"rtol 1e-6{', the 256^3 selection workload and its adjoint at rtol 1e-6' if full else ''})",
            "time_to_map": ttm}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--hvp-reps", type=int, default=200)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-full", action="store_true",
                    help="CPU oracle baseline at full size: 256^3 solves and adjoint, all 64 batch instances "
                         "(minutes of host CPU)")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched workload")
    ap.add_argument("--only-hvp", action="store_true", help="profiling aid: only the isolated HVP loop")
    ap.add_argument("--only-batch", action="store_true", help="profiling aid: only the batched workload")
    ap.add_argument("--only-solve", action="store_true",
                    help="profiling aid: only the timed FP64 and mixed MAP solves (no isolated HVP loop)")
    ap.add_argument("--only-cpu", action="store_true",
                    help="only the CPU oracle baseline (host cores, no GPU); with --cpu-full the full-size one")
    ap.add_argument("--n", type=int, default=None, help="override the grid length (same cell size)")
    ap.add_argument("--workload", default="sel256", choices=["sel256", "bias256", "big512"],
                    help="sel256: 256^3 selection workload (default); bias256: beta = 1.5, nbar = 2 "
                         "(forward + adjoint); big512: 512^3, sigma_G = 2, beta = 1.2")
    ap.add_argument("--copy-probe", action="store_true",
                    help="profiling aid: also run a 1 GiB device-to-device copy (counter scale reference)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build runs on exactly one GPU (the solver is single-GPU); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    if args.only_cpu:
        from paper_0911_1407_amd import synth
        inst = synth.config_instance(args.workload, n=args.n)
        v = np.random.default_rng([0, 3]).standard_normal(inst["n"])
        print(json.dumps(cpu_oracle_baseline(inst, v, full=args.cpu_full)))
        return

    import torch
    from paper_0911_1407_amd import synth
    from paper_0911_1407_amd.binding import Plan

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.only_batch:
        print(json.dumps(batched_workload(dev, 1e-6)))
        return
    t0 = time.time()
    inst = synth.config_instance(args.workload, n=args.n)
    print(f"# generated inputs n={inst['n']} in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    n = inst["n"]
    rtol = 1e-6

    plan = Plan(n, inst["box"], precision="mixed", device=dev)
    plan.set_instance(inst)
    variants = plan.autotune(TUNE_CACHE if os.path.exists(TUNE_CACHE) else None)
    print(f"# tile variants {variants}", file=sys.stderr, flush=True)
    s_true = torch.from_numpy(inst["s_true"]).to(dev)
    mu = float(inst["mu"])

    out = {}
    # ---------------- isolated HVP (roofline) ----------------
    plan.grad(s_true)  # linearise at s_true: caches d
    rng = np.random.default_rng([0, 3])
    v = rng.standard_normal(n)
    v_hat64 = torch.from_numpy(np.fft.rfftn(v)).to(dev)
    v_hat32 = v_hat64.to(torch.complex64)
    hv64 = torch.empty_like(v_hat64)
    hv32 = torch.empty_like(v_hat32)
    stream = torch.cuda.current_stream(dev)

    def time_hvp(vin, vout, reps):
        # 20 warm-up calls, then `reps` back-to-back calls, each bracketed by
        # HIP events on the plan's stream; the median per-call time
        for _ in range(20):
            plan.hessvec_hat(vin, out=vout)
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
        ev[0].record(stream)
        for i in range(reps):
            plan.hessvec_hat(vin, out=vout)
            ev[i + 1].record(stream)
        torch.cuda.synchronize()
        per_call = sorted(ev[i].elapsed_time(ev[i + 1]) for i in range(reps))
        return float(np.median(per_call))  # ms per HVP

    if not args.only_solve:
        ms64 = time_hvp(v_hat64, hv64, args.hvp_reps)
        ms32 = time_hvp(v_hat32, hv32, args.hvp_reps)
        b64 = hvp_bytes(n, 8)
        b32 = hvp_bytes(n, 4)
        gbs64 = b64 / (ms64 * 1e-3) / 1e9
        gbs32 = b32 / (ms32 * 1e-3) / 1e9
        print(f"# HVP fp64 {ms64:.3f} ms ({gbs64:.0f} GB/s), fp32 {ms32:.3f} ms ({gbs32:.0f} GB/s)",
              file=sys.stderr, flush=True)
        if args.copy_probe:
            src = torch.empty(1 << 27, dtype=torch.float64, device=dev).fill_(1.0)
            dst = torch.empty_like(src)
            for _ in range(3):
                dst.copy_(src)
            torch.cuda.synchronize()
        if args.only_hvp:
            print(json.dumps({"hvp_ms_fp64": ms64, "hvp_ms_fp32": ms32}))
            return

    # ---------------- timed FP64 solves (the steps) ----------------
    s = torch.empty(n, dtype=torch.float64, device=dev)

    def one_solve(precision):
        s.fill_(mu)
        from paper_0911_1407_amd.binding import make_opts, pl_newton_krylov_solve
        info = pl_newton_krylov_solve(plan.h, s, make_opts(rtol=rtol, precision=precision))
        return info.as_dict()

    for _ in range(args.warmup):
        one_solve(0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = [one_solve(0) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t_fp64 = time.perf_counter() - t0
    hvps = sum(i["hvps"] for i in infos)
    for i in infos:
        if i["status"] != 0:
            print(f"# WARNING solve status {i}", file=sys.stderr)
    ms_per_step = 1e3 * t_fp64 / args.steps
    value = hvps / t_fp64
    print(f"# fp64 solve {ms_per_step:.1f} ms, {infos[-1]}", file=sys.stderr, flush=True)

    # ---------------- mixed-precision solves ----------------
    one_solve(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    minfos = [one_solve(1) for _ in range(max(1, args.steps))]
    torch.cuda.synchronize()
    t_mixed = (time.perf_counter() - t0) / max(1, args.steps)
    s_mixed = s.clone()
    one_solve(0)
    s_fp64 = s.clone()
    mixed_rel = float(torch.linalg.norm(s_mixed - s_fp64) / torch.linalg.norm(s_fp64))
    print(f"# mixed solve {1e3 * t_mixed:.1f} ms, {minfos[-1]}, rel vs fp64 {mixed_rel:.2e}",
          file=sys.stderr, flush=True)
    if args.only_solve:
        print(json.dumps({"fp64_ms": ms_per_step, "fp64": infos[-1], "hvp_per_s": value,
                          "mixed_ms": 1e3 * t_mixed, "mixed": minfos[-1]}))
        return
    parity = oracle_parity(args.workload if args.n is None else None, inst,
                           {"fp64_rtol_1e-6": s_fp64, "mixed_rtol_1e-6": s_mixed})
    if parity:
        print(f"# rel-L2 vs the stored oracle MAP: {parity}", file=sys.stderr, flush=True)

    # ---------------- adjoint at the MAP ----------------
    dL = 2.0 * (s_fp64 - s_true)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    grads, ainfo = plan.adjoint(s_fp64, dL, want_fields=False, rtol=1e-6, precision=0, max_cg=20000)
    torch.cuda.synchronize()
    t_adj = time.perf_counter() - t0
    t0 = time.perf_counter()
    grads32, ainfo32 = plan.adjoint(s_fp64, dL, want_fields=False, rtol=1e-6, precision=1, max_cg=20000)
    torch.cuda.synchronize()
    t_adj32 = time.perf_counter() - t0
    adj_agree = {k: abs(grads32[k] - grads[k]) / abs(grads[k]) for k in ("A", "beta", "nbar") if grads[k] != 0.0}
    print(f"# adjoint fp64 {1e3 * t_adj:.1f} ms {ainfo}; mixed {1e3 * t_adj32:.1f} ms, "
          f"mixed vs fp64 {adj_agree}", file=sys.stderr, flush=True)

    # ---------------- the 32^3 plain workload (time-to-MAP beside the oracle's) ----------------
    small = synth.config_instance("plain32")
    splan = Plan(small["n"], small["box"], precision="mixed", device=dev)
    splan.set_instance(small)
    splan.autotune(TUNE_CACHE if os.path.exists(TUNE_CACHE) else None)
    plain32 = {}
    for name, prec in (("fp64", 0), ("mixed", 1)):
        splan.solve(rtol=1e-8, precision=prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s32, sinfo = splan.solve(rtol=1e-8, precision=prec)
        torch.cuda.synchronize()
        plain32[name] = {"ms": 1e3 * (time.perf_counter() - t0), "newton_its": sinfo["newton_its"],
                         "cg_its": sinfo["cg_its"], "status": sinfo["status"], "fp64_steps": sinfo["fp64_steps"],
                         "oracle_parity": oracle_parity("plain32", small, {"s": s32})}
    splan.close()
    print(f"# plain32 (rtol 1e-8): {plain32}", file=sys.stderr, flush=True)

    # ---------------- paper-literal Krylov step (nonlinear-CG search vectors) ----------------
    s_nl, ninfo = plan.solve_nlcg(rtol=rtol, max_cg=20000)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s_nl, ninfo = plan.solve_nlcg(rtol=rtol, max_cg=20000)
    torch.cuda.synchronize()
    t_nlcg = time.perf_counter() - t0
    nlcg_rel = float(torch.linalg.norm(s_nl - s_fp64) / torch.linalg.norm(s_fp64))
    nlcg = {"ms": 1e3 * t_nlcg, "steps": ninfo["cg_its"], "hvps": ninfo["hvps"], "status": ninfo["status"],
            "rel_grad": ninfo["rel_grad"], "rel_l2_vs_newton_krylov": nlcg_rel,
            "time_vs_newton_krylov": 1e3 * t_nlcg / ms_per_step}
    print(f"# nlcg fp64 {1e3 * t_nlcg:.1f} ms, {ninfo['cg_its']} steps, rel vs Newton-Krylov {nlcg_rel:.2e}",
          file=sys.stderr, flush=True)

    # ---------------- comparison estimators (section 4.1) ----------------
    # LSQ-Wiener filter (FP64 and refined mixed), inverse weighting, and the
    # correlation coefficient / Euclidean distance of each reconstruction
    # against the true overdensity exp(s_true) - 1
    plan.lsq(rtol=rtol, max_cg=20000, precision=0)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    d_lsq, linfo = plan.lsq(rtol=rtol, max_cg=20000, precision=0)
    torch.cuda.synchronize()
    t_lsq = time.perf_counter() - t0
    t0 = time.perf_counter()
    d_lsq32, linfo32 = plan.lsq(rtol=rtol, max_cg=20000, precision=1)
    torch.cuda.synchronize()
    t_lsq32 = time.perf_counter() - t0
    # Gaussian-prior MAP (eq. MAPG), FP64
    plan.solve_gaussian(rtol=rtol, max_newton=200, max_cg=20000)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    d_gauss, ginfo = plan.solve_gaussian(rtol=rtol, max_newton=200, max_cg=20000)
    torch.cuda.synchronize()
    t_gauss = time.perf_counter() - t0
    d_true = torch.expm1(s_true)
    quality = {}
    for name, rec in (("lognormal_map", torch.expm1(s_fp64)), ("gaussian_map", d_gauss), ("lsq_wiener", d_lsq),
                      ("inverse_weighting", plan.inverse_weight())):
        r, dist = plan.compare(rec, d_true)
        quality[name] = {"r": r, "d_euc": dist}
    # lognormal prior from a matter spectrum (section 2.3), the workload's
    # spectrum and amplitude read as the matter spectrum
    pk_dev = torch.from_numpy(inst["pk"]).to(dev)
    plan.lognormal_prior(pk_dev, inst["amp"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, pinfo = plan.lognormal_prior(pk_dev, inst["amp"])
    torch.cuda.synchronize()
    t_prior = time.perf_counter() - t0
    estimators = {"lognormal_prior_ms": 1e3 * t_prior, "lognormal_prior": pinfo,
                  "gaussian_map_ms_fp64": 1e3 * t_gauss, "gaussian_map_newton_its": ginfo["newton_its"],
                  "gaussian_map_cg_its": ginfo["cg_its"], "gaussian_map_status": ginfo["status"],
                  "lsq_ms_fp64": 1e3 * t_lsq, "lsq_ms_mixed": 1e3 * t_lsq32, "lsq_cg_its_fp64": linfo["cg_its"],
                  "lsq_cg_its_mixed": linfo32["cg_its"], "quality_vs_true_overdensity": quality}
    print(f"# lsq fp64 {1e3 * t_lsq:.1f} ms ({linfo['cg_its']} its), mixed {1e3 * t_lsq32:.1f} ms "
          f"({linfo32['cg_its']} its); quality {quality}", file=sys.stderr, flush=True)

    # ---------------- linear (non-local) bias (sections 2.2.1, 2.4.1) ----------------
    # b_hat(k) = exp(-(1.5 cells k)^2 / 2): the galaxy field as the matter
    # field smoothed over 1.5 cells; both priors, FP64, same tolerance
    # (selection workload at its own size only)
    linear_bias = None
    lb_models = (("lognormal", s_true), ("gaussian", torch.expm1(s_true)))
    if args.workload != "sel256" or args.n is not None:
        lb_models = ()
    else:
        cell = inst["box"][0] / n[0]
        bk = torch.from_numpy(synth.bias_multiplier_half(n, inst["box"], 1.0, 1.5 * cell)).to(dev)
        linear_bias = {"b_hat": "exp(-(1.5 cells * k)^2 / 2)"}
        v_real = torch.from_numpy(v).to(dev)
        hv_real = torch.empty_like(v_real)
    for model, x_lin in lb_models:
        plan.linear_bias_grad(model, bk, x_lin)
        for _ in range(5):
            plan.linear_bias_hessvec(model, bk, v_real, out=hv_real)
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(21)]
        ev[0].record(stream)
        for i in range(20):
            plan.linear_bias_hessvec(model, bk, v_real, out=hv_real)
            ev[i + 1].record(stream)
        torch.cuda.synchronize()
        ms_lb = float(np.median(sorted(ev[i].elapsed_time(ev[i + 1]) for i in range(20))))
        bytes_lb = linear_bias_hvp_bytes(n, model == "lognormal")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x_lb, lbinfo = plan.solve_linear_bias(model, bk, rtol=rtol, max_newton=200, max_cg=20000)
        torch.cuda.synchronize()
        t_lb = time.perf_counter() - t0
        linear_bias[model] = {"solve_ms_fp64": 1e3 * t_lb, "newton_its": lbinfo["newton_its"],
                              "cg_its": lbinfo["cg_its"], "hvps": lbinfo["hvps"], "status": lbinfo["status"],
                              "rel_grad": lbinfo["rel_grad"], "hvp_real_ms": ms_lb,
                              "hvp_real_bytes": bytes_lb, "hvp_real_gbs": bytes_lb / (ms_lb * 1e-3) / 1e9}
        print(f"# linear bias {model}: solve {1e3 * t_lb:.1f} ms ({lbinfo['newton_its']} Newton, "
              f"{lbinfo['cg_its']} CG, status {lbinfo['status']}), real-space HVP {ms_lb:.3f} ms "
              f"({bytes_lb / (ms_lb * 1e-3) / 1e9:.0f} GB/s)", file=sys.stderr, flush=True)

    # ---------------- batched workload ----------------
    batch = None
    if not args.no_batch and args.workload == "sel256" and args.n is None:
        batch = batched_workload(dev, rtol)

    # ---------------- CPU oracle baseline ----------------
    cpu = None
    if not args.no_cpu:
        cpu = cpu_oracle_baseline(inst, v, args.cpu_full)
        print(f"# cpu oracle HVP {1e3 / cpu['value']:.0f} ms; {json.dumps(cpu['time_to_map'])}",
              file=sys.stderr, flush=True)

    wl_desc = {
        "sel256": "selection workload (sigma_G 1.5, w=exp(-(r/R)^2) x 20% masked 8^3 blocks, nbar 0.5, beta 1)",
        "bias256": "bias workload (sigma_G 1.5, selection and mask as sel256, nbar 2, beta 1.5)",
        "big512": "512^3 workload (sigma_G 2, w=exp(-(r/400)^2), nbar 0.2, beta 1.2)",
    }[args.workload]
    result = {
        "metric": "Hessian-vector products/sec at 256^3 (%HBM peak); time-to-MAP + adjoint vs plain FP64",
        "value": value,
        "unit": "HVP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{n[0]}^3 {wl_desc}, box {inst['box'][0]:.0f} Mpc/h; "
                               f"FP64 Newton-Krylov MAP to rtol {rtol:g}",
                   "grid": list(n), "rtol": rtol, "tile_variants": variants},
        "roofline": {"bound": "hbm", "achieved": gbs64, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": gbs64 / HBM_PEAK_GBS,
                     "traffic": measured_traffic(args.workload, variants["fp64"]) if args.n is None else None,
                     "traffic_unit": "bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-scaled)",
                     "kernel": "spectral HVP (5 passes), FP64", "bytes_per_launch": b64,
                     "ms_per_launch": ms64},
        "hvp_fp32": {"achieved": gbs32, "frac": gbs32 / HBM_PEAK_GBS, "bytes_per_launch": b32,
                     "ms_per_launch": ms32, "hvp_per_s": 1e3 / ms32},
        "hvp_fp64_per_s_isolated": 1e3 / ms64,
        "solve_fp64": {"ms": ms_per_step, "newton_its": infos[-1]["newton_its"],
                       "cg_its": infos[-1]["cg_its"], "hvps": infos[-1]["hvps"],
                       "rel_grad": infos[-1]["rel_grad"]},
        "solve_mixed": {"ms": 1e3 * t_mixed, "newton_its": minfos[-1]["newton_its"],
                        "cg_its": minfos[-1]["cg_its"], "hvps": minfos[-1]["hvps"],
                        "rel_grad": minfos[-1]["rel_grad"], "speedup_vs_fp64": ms_per_step / (1e3 * t_mixed),
                        "rel_l2_vs_fp64": mixed_rel, "fp64_steps": minfos[-1]["fp64_steps"]},
        "oracle_parity": parity,
        "adjoint": {"ms_fp64": 1e3 * t_adj, "ms_mixed": 1e3 * t_adj32, "cg_its_fp64": ainfo["cg_its"],
                    "cg_its_mixed": ainfo32["cg_its"], "dL_dA": grads["A"], "dL_dbeta": grads["beta"],
                    "dL_dnbar": grads["nbar"], "mixed_vs_fp64_rel": adj_agree},
        "plain32_time_to_map": plain32,
        "nlcg": nlcg,
        "estimators": estimators,
        "linear_bias": linear_bias,
        "batched": batch,
        "cpu_baseline": cpu,
    }
    print(json.dumps(result))


if __name__ == "__main__":
    main()
