#!/usr/bin/env python3
"""Benchmark of the MPS-LCC hot path on one MI355X: the two-site H_eff x and the local LCC
solve (conjugate gradients, Implementation section), mixed precision against FP64.

A step is one local LCC solve Q(H_eff - E0)Q x = Q b from x = 0 to a relative FP64 residual
of 1e-10, with the low-precision operator inside FP64 iterative refinement, on environments
already resident in HBM.  `value` is the H_eff x throughput sustained inside those solves:
(algorithmic flops per H_eff x) x (number of H_eff x products of all precisions) / time.

Prints one JSON line.  Only one GPU is used.
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

PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16": 2500.0}
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def shift_for(spec, env, name):
    """E0 that makes Q(H_eff - E0)Q positive definite (see workloads.configs)."""
    from workloads import configs as C
    if spec["eri"] is None:
        return C.lower_bound_shift(spec, 0.5), "E(U=0) - 0.5"
    theta, res = env.lowest_eigenvalue(steps=60, seed=7)
    return theta - max(0.5, 2.0 * res), f"lanczos theta={theta:.12f} res={res:.3e}, minus max(0.5, 2 res)"


def source_digest() -> str:
    """sha1 of the sources that determine the GEMM kernels and the plan they run."""
    import hashlib
    h = hashlib.sha1()
    for f in ("kernels.hip", "env.cpp", "internal.h", "tune.cpp"):
        with open(os.path.join(ROOT, "paper_1509_00216_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def kernel_name(precision: str, launch: dict) -> str:
    if launch["kind"] == "reduce":
        return "reduce_kernel<%s>" % ("double" if precision == "fp64" else "float")
    ta = "true" if launch["a_kmajor"] else "false"
    tb = "true" if launch["b_colmajor"] else "false"
    bm, bn = launch["tile"]
    waves = {(64, 64): (2, 2), (16, 64): (1, 4), (64, 16): (4, 1), (32, 32): (2, 2), (128, 64): (2, 2),
             (64, 128): (2, 2), (32, 64): (2, 2), (64, 32): (2, 2)}[(bm, bn)]
    kind = "packed" if launch.get("packed") else "terms"
    if precision == "bf16x3":
        return f"gemm_bf16x3_{kind}_kernel<{ta}, {tb}, {bm}, {bn}, {waves[0]}, {waves[1]}>"
    mode = 0 if precision == "fp64" else 1
    return f"gemm_{kind}_kernel<{mode}, {ta}, {tb}, {bm}, {bn}, {waves[0]}, {waves[1]}>"


def measured_traffic(kname: str, tiles: int, workload: str):
    """HBM bytes per launch of `kname` with `tiles` workgroups from the committed PMC summary, if
    the kernel sources have not changed since the counters were taken (else None)."""
    path = os.path.join(ROOT, "profiles", f"pmc_traffic_{workload}.txt")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
    except Exception:
        return None
    if rec.get("source_sha1") != source_digest():
        return None
    ent = rec.get("kernels", {}).get(f"{kname} x{tiles}")
    return None if ent is None else ent.get("traffic_bytes")


def cpu_baseline(sample_seconds_target=20.0):
    """The oracle (plain numpy FP64, prefix-automaton MPO) on a bounded sample of the ab initio
    family, with the product's algorithmic flop count of the same H_eff x as the work unit."""
    import torch
    from oracle import blocksparse as BS
    from oracle import mpo as OM
    from paper_1509_00216_amd import lcc
    from workloads import hamiltonians as H
    from workloads import mps as M
    spec = H.random_ab_initio(10, 6, seed=1003)
    mps = M.random_mps(10, 6, 0, 60, seed=1003)
    ctx = lcc.Context(0)
    env = ctx.build_environments(ctx.create_hamiltonian(spec), mps)
    flops = env.flops_per_apply
    env.close()
    t0 = time.perf_counter()
    oenv = BS.Environments(spec, mps, OM.build_mpo(spec))
    t_setup = time.perf_counter() - t0
    x = M.random_two_site_vector(mps, 5)
    reps, t_apply = 0, 0.0
    while t_apply < sample_seconds_target and reps < 50:
        t0 = time.perf_counter()
        oenv.apply(x)
        t_apply += time.perf_counter() - t0
        reps += 1
    try:
        threads = torch.get_num_threads()
    except Exception:
        threads = os.cpu_count()
    return {
        "value": flops * reps / t_apply / 1e9,
        "unit": "GFLOP/s",
        "cores": int(os.environ.get("OMP_NUM_THREADS", threads) or threads),
        "kind": "oracle",
        "sample": (f"oracle block-sparse H_eff x, ab initio K=10 N=6 M=60 (the K=24 M=1000 environments "
                   f"exceed the oracle's prefix-automaton MPO), {reps} applies in {t_apply:.1f}s after "
                   f"{t_setup:.1f}s setup; work = the plan's {flops:.3e} algorithmic flops per apply"),
    }


SHIPPED_TUNE_CACHE = os.path.join(ROOT, "paper_1509_00216_amd", "tune_cache.txt")


def working_tune_cache(path: str) -> str:
    """A private copy of the tuning cache (entries found by this run are appended there, the
    shipped file is left as it is)."""
    import shutil
    import tempfile
    fd, tmp = tempfile.mkstemp(prefix="lcc_tune_", suffix=".txt")
    os.close(fd)
    if path and os.path.exists(path):
        shutil.copyfile(path, tmp)
    return tmp


def run_tune(args):
    """Autotune the named workloads' environments and append the results to --tune-cache."""
    import torch
    from paper_1509_00216_amd import lcc
    from workloads import configs as C
    torch.cuda.init()
    for name in args.tune_workloads.split(","):
        spec, mps = C.make(name)
        ctx = lcc.Context(0)
        ctx.set_tune_cache(args.tune_cache)
        env = ctx.build_environments(ctx.create_hamiltonian(spec), mps)
        info = env.autotune("fp32", reps=5)
        print(json.dumps({"mode": "tune", "workload": name, **info}), flush=True)
        env.close()


def run_batch(args):
    """64 independent local problems (ab initio K=24, 4x4 Hubbard, 3-band cluster; M uniform in
    [128, 1500], jittered sector weights): one batched mixed-precision solve (merged launches,
    graph-replayed iterations) against the 64 problems solved one after another in FP64."""
    import torch
    from paper_1509_00216_amd import lcc
    from workloads import configs as C
    from workloads import mps as M
    torch.cuda.init()
    dev = torch.device("cuda:0")
    ctx = lcc.Context(0)
    ctx.set_intermediate_limit(args.batch_intermediate_mib << 20)
    members = C.batch_members(args.batch_n)
    envs, bs, e0s, flops = [], [], [], []
    hams = {}
    t0 = time.perf_counter()
    for i, (parent, m, seed) in enumerate(members):
        spec, mps = C.make_member(parent, m, seed)
        if parent not in hams:
            hams[parent] = ctx.create_hamiltonian(spec)
        env = ctx.build_environments(hams[parent], mps)
        e0, _ = shift_for(spec, env, parent)
        envs.append(env)
        e0s.append(e0)
        flops.append(env.flops_per_apply)
        bs.append(torch.tensor(env.pack(M.random_two_site_vector(mps, seed + 7)), dtype=torch.float64, device=dev))
        log(f"[batch] member {i}: {parent} M={m} n={env.n} F={env.flops_per_apply:.3e} E0={e0:.6f}")
    t_setup = time.perf_counter() - t0
    xs = [torch.zeros_like(b) for b in bs]
    batch = lcc.Batch(ctx, envs)
    status, infos = batch.solve(bs, e0s, xs, precision=args.precision, tol=1e-10, max_iter=5000,
                                inner_tol=args.inner_tol)  # warm-up
    torch.cuda.synchronize()
    reps = max(1, args.steps)
    t0 = time.perf_counter()
    for _ in range(reps):
        for x in xs:
            x.zero_()
        status, infos = batch.solve(bs, e0s, xs, precision=args.precision, tol=1e-10, max_iter=5000,
                                    inner_tol=args.inner_tol)
    torch.cuda.synchronize()
    ms_batch = (time.perf_counter() - t0) * 1e3 / reps
    # sequential FP64 baseline on the same problems
    seq = []
    x1 = [torch.zeros_like(b) for b in bs]
    envs[0].solve_local_lcc(bs[0], e0s[0], x1[0], precision="fp64", tol=1e-10, max_iter=5000)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for env, b, e0, x in zip(envs, bs, e0s, x1):
        x.zero_()
        seq.append(env.solve_local_lcc(b, e0, x, precision="fp64", tol=1e-10, max_iter=5000))
    torch.cuda.synchronize()
    ms_seq = (time.perf_counter() - t0) * 1e3
    dE = [abs(a["hylleraas"] - b["hylleraas"]) for a, b in zip(infos, seq)]
    applies = sum(i["applies_fp64"] + i["applies_low"] for i in infos) / len(infos)
    out = {"mode": "batch", "problems": len(envs), "precision": args.precision, "status": status,
           "ms_batched_mixed": ms_batch, "ms_sequential_fp64": ms_seq, "speedup": ms_seq / ms_batch,
           "max_energy_diff": max(dE), "max_rel_residual": max(i["rel_residual"] for i in infos),
           "mean_applies_per_problem": applies, "flops_per_apply_total": sum(flops),
           "gflops_batched": sum(f * (i["applies_fp64"] + i["applies_low"]) for f, i in zip(flops, infos)) /
           (ms_batch * 1e-3) / 1e9,
           "setup_s": t_setup, "intermediate_limit_mib": args.batch_intermediate_mib,
           "members": [{"parent": p, "m": m} for p, m, _ in members]}
    print(json.dumps(out), flush=True)


def run_sweep(args):
    """One left-to-right sweep of two-site local solves over the 4x4 Hubbard model (K=16,
    M=500): solve, SVD split, truncation, left-environment update, next guess; FP64 solves
    against mixed-precision solves (separate sweeps from the same start)."""
    import torch
    from paper_1509_00216_amd import lcc
    from workloads import configs as C
    from workloads import mps as M
    torch.cuda.init()
    dev = torch.device("cuda:0")
    name = "hubbard2d_4x4_m500"
    spec, mps = C.make(name, center=0)
    e0 = C.lower_bound_shift(spec, 0.5)
    ctx = lcc.Context(0)
    ctx.set_tune_cache(working_tune_cache(args.tune_cache))
    ham = ctx.create_hamiltonian(spec)
    m_max = C.WORKLOADS[name][1]
    out = {"mode": "sweep", "workload": name, "m_max": m_max, "e0": e0}
    for prec in ("fp64", args.precision):
        sw = lcc.Sweep(ctx, ham, mps, 0)
        env = sw.env()
        b = torch.tensor(env.pack(M.random_two_site_vector(mps, 77)), dtype=torch.float64, device=dev)
        sites = []
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        t_solve = 0.0
        for l in range(spec["n_orb"] - 1):
            x = torch.zeros_like(b)
            t0 = time.perf_counter()
            info = env.solve_local_lcc(b, e0, x, precision=prec, tol=1e-10, max_iter=5000, inner_tol=args.inner_tol,
                                       max_outer=200)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            t_solve += dt
            rec = {"site": l, "n": env.n, "ms": dt * 1e3, "iterations": info["iterations"], "J": info["hylleraas"],
                   "status": info["status"]}
            if l + 1 < spec["n_orb"] - 1:
                split = sw.advance(x, m_max)
                rec["kept"] = split["kept"]
                rec["discarded_weight"] = split["discarded_weight"]
                rec["advance_ms"] = {k: split[k] for k in ("ms_svd", "ms_env", "ms_guess", "ms_total")}
                env = sw.env()
                b = torch.empty(env.n, dtype=torch.float64, device=dev)
                sw.guess(b)
                b /= b.norm()
            sites.append(rec)
        torch.cuda.synchronize()
        out[prec] = {"sweep_ms": (time.perf_counter() - t_start) * 1e3, "solve_ms": t_solve * 1e3, "sites": sites}
        sw.close()
        log(f"[sweep] {prec}: {out[prec]['sweep_ms']:.1f} ms")
    a, b2 = out["fp64"]["sites"], out[args.precision]["sites"]
    out["max_J_diff"] = max(abs(x["J"] - y["J"]) for x, y in zip(a, b2))
    out["speedup_solves"] = out["fp64"]["solve_ms"] / out[args.precision]["solve_ms"]
    out["speedup_sweep"] = out["fp64"]["sweep_ms"] / out[args.precision]["sweep_ms"]
    print(json.dumps(out), flush=True)



def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="abinitio_k24_m1000")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16x3"])
    ap.add_argument("--apply-reps", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-solve", action="store_true")
    ap.add_argument("--apply-only", type=int, default=0, metavar="N",
                    help="profiling mode: build, run N plain H_eff x products of --apply-precision and a "
                         "256 MiB device copy (counter calibration), print timings, skip the solves")
    ap.add_argument("--apply-precision", default="fp32", choices=["fp64", "fp32", "bf16x3"])
    ap.add_argument("--mode", default="solve", choices=["solve", "batch", "sweep", "tune"],
                    help="solve: the headline local solve (default); batch: 64 independent problems, batched "
                         "mixed vs sequential FP64; sweep: one sweep of the 4x4 Hubbard model; tune: autotune "
                         "--tune-workloads into --tune-cache")
    ap.add_argument("--tune-cache", default=SHIPPED_TUNE_CACHE)
    ap.add_argument("--tune-workloads", default="abinitio_k24_m1000,threeband_4x2_m2000,hubbard2d_4x4_m500")
    ap.add_argument("--no-tune", action="store_true", help="plan with the default planner parameters")
    ap.add_argument("--inner-tol", type=float, default=1e-4,
                    help="mixed precision: residual reduction between FP64 refreshes")
    ap.add_argument("--batch-n", type=int, default=64)
    ap.add_argument("--batch-intermediate-mib", type=int, default=1024)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (--gpus must be 1)", file=sys.stderr)
        sys.exit(2)

    if args.mode == "tune":
        return run_tune(args)
    if args.mode == "batch":
        return run_batch(args)
    if args.mode == "sweep":
        return run_sweep(args)

    import torch
    from paper_1509_00216_amd import lcc
    from workloads import configs as C
    from workloads import mps as M

    torch.cuda.init()
    dev = torch.device("cuda:0")
    log(f"[bench] workload {args.workload}: generating inputs")
    spec, mps = C.make(args.workload)
    ctx = lcc.Context(0)
    if not args.no_tune:
        ctx.set_tune_cache(working_tune_cache(args.tune_cache))
    t0 = time.perf_counter()
    ham = ctx.create_hamiltonian(spec)
    t_ham = time.perf_counter() - t0
    log(f"[bench] MPO built in {t_ham:.2f}s; building environments")
    t0 = time.perf_counter()
    env = ctx.build_environments(ham, mps)
    t_env = time.perf_counter() - t0
    f1, f2 = env.flops()
    F = f1 + f2
    log(f"[bench] environments in {t_env:.2f}s: n={env.n} D_mid={env.mpo_bond_dim} F_alg={F:.4e} (phase1 {f1:.3e}, phase2 {f2:.3e})")
    tune = None
    if not args.no_tune:
        t0 = time.perf_counter()
        tune = env.autotune("fp32", reps=3)
        tune["seconds"] = time.perf_counter() - t0
        log(f"[bench] plan: {tune}")
    if args.apply_only > 0:
        prec = args.apply_precision
        xx = torch.tensor(env.pack(M.random_two_site_vector(mps, 17)), dtype=torch.float64, device=dev)
        if prec != "fp64":
            xx = xx.float()
        yy = torch.empty_like(xx)
        src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device=dev)  # 256 MiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        env.apply_heff(xx, yy, prec)  # warm-up (and the lazily built FP32 environments)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(args.apply_only):
            env.apply_heff(xx, yy, prec)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / args.apply_only
        print(json.dumps({"mode": "apply-only", "workload": args.workload, "precision": prec, "applies": args.apply_only,
                          "ms_per_apply": ms, "flops_per_apply": F, "phase1_flops": f1, "phase2_flops": f2,
                          "gflops": F / (ms * 1e-3) / 1e9, "copy_bytes": src.numel() * 8}), flush=True)
        return
    e0, e0_rule = shift_for(spec, env, args.workload)
    log(f"[bench] E0 = {e0:.12f} ({e0_rule})")

    # --- per-precision H_eff x throughput (HIP events around each phase, on the context stream)
    applies = {}
    x64 = torch.tensor(env.pack(M.random_two_site_vector(mps, 17)), dtype=torch.float64, device=dev)
    for prec in ("fp64", "fp32", "bf16x3"):
        xx = x64 if prec == "fp64" else x64.float()
        yy = torch.empty_like(xx)
        env.profile_apply(xx, yy, prec, reps=1)  # warm-up (and FP32 environment copies)
        ms1, ms2 = env.profile_apply(xx, yy, prec, reps=args.apply_reps)
        # wall time of lcc_apply_heff as the solver calls it (launches of a phase concurrent)
        env.apply_heff(xx, yy, prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.apply_reps):
            env.apply_heff(xx, yy, prec)
        torch.cuda.synchronize()
        ms_wall = (time.perf_counter() - t0) * 1e3 / args.apply_reps
        applies[prec] = {"ms_phase1": ms1, "ms_phase2": ms2, "ms": ms1 + ms2, "ms_wall": ms_wall,
                         "gflops": F / (ms_wall * 1e-3) / 1e9}
        log(f"[bench] apply {prec}: phase1 {ms1:.3f} ms, phase2 {ms2:.3f} ms (launches in order), "
            f"{ms_wall:.3f} ms wall, {applies[prec]['gflops']:.1f} GFLOP/s")

    # --- timed steps: mixed-precision local solves from x = 0
    b = torch.tensor(env.pack(M.random_two_site_vector(mps, 2025)), dtype=torch.float64, device=dev)
    x = torch.zeros_like(b)

    def solve(prec):
        x.zero_()
        return env.solve_local_lcc(b, e0, x, precision=prec, tol=1e-10, max_iter=5000, inner_tol=args.inner_tol,
                                   max_outer=200)

    for i in range(args.warmup):
        info = solve(args.precision)
        log(f"[bench] warmup {i}: {info}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    for i in range(args.steps):
        infos.append(solve(args.precision))
        log(f"[bench] step {i}: {infos[-1]}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_step = elapsed * 1e3 / args.steps
    n_app = sum(i["applies_fp64"] + i["applies_low"] for i in infos)
    value = F * n_app / elapsed / 1e9
    j_mixed = infos[-1]["hylleraas"]

    fp64 = None
    if not args.no_fp64_solve:
        t0 = time.perf_counter()
        info64 = solve("fp64")
        torch.cuda.synchronize()
        fp64 = {"ms": (time.perf_counter() - t0) * 1e3, "iterations": info64["iterations"],
                "hylleraas": info64["hylleraas"], "status": info64["status"]}
        log(f"[bench] fp64 solve: {info64}")

    # --- roofline of the dominant kernel launch of the timed precision (HIP events per launch)
    xx = x64 if args.precision == "fp64" else x64.float()
    yy = torch.empty_like(xx)
    launches = env.profile_launches(xx, yy, args.precision, reps=args.apply_reps)
    dom = max(launches, key=lambda r: r["ms"])
    mult = 3.0 if args.precision == "bf16x3" else 1.0
    peak = PEAK_TFLOPS["bf16" if args.precision == "bf16x3" else "fp32"]
    achieved = mult * dom["flops"] / (dom["ms"] * 1e-3) / 1e12
    kname = kernel_name(args.precision, dom)
    roofline = {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
                "traffic": measured_traffic(kname, dom["n_tiles"], args.workload), "kernel": kname,
                "launch_ms": dom["ms"], "launch_flops": dom["flops"], "launch_algorithmic_bytes": dom["bytes"],
                "launch_tiles": dom["n_tiles"],
                "launches_per_apply": len(launches),
                "note": ("bf16x3 counts the three bf16 MFMA products per algorithmic flop" if mult == 3.0 else
                         "achieved = the launch's algorithmic flops / its mean HIP-event duration")}

    out = {
        "metric": "H_eff·x GFLOP/s + local LCC solve ms at M=1000, mixed vs FP64, 1 MI355X",
        "value": value,
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if args.precision == "fp32" else "bf16x3+f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "n_orb": spec["n_orb"], "n_elec": spec["n_elec"],
                   "two_sz": spec["two_sz"], "m_max": C.WORKLOADS[args.workload][1], "site": mps["center"],
                   "vector_elements": env.n, "mpo_bond_dim_mid": env.mpo_bond_dim, "flops_per_apply": F,
                   "parallelism": "single GPU"},
        "solve": {"precision": args.precision, "inner_tol": args.inner_tol or 0.1, "ms": ms_step, "iterations": infos[-1]["iterations"],
                  "outer": infos[-1]["outer"], "applies_fp64": infos[-1]["applies_fp64"],
                  "applies_low": infos[-1]["applies_low"], "hylleraas": j_mixed,
                  "rel_residual": infos[-1]["rel_residual"], "e0": e0,
                  "fp64": fp64, "energy_diff_vs_fp64": (abs(j_mixed - fp64["hylleraas"]) if fp64 else None),
                  "speedup_vs_fp64": (fp64["ms"] / ms_step if fp64 else None)},
        "apply": {p: {"gflops": v["gflops"], "ms": v["ms_wall"], "ms_launches_in_order": v["ms"],
                      "ms_phase1": v["ms_phase1"], "ms_phase2": v["ms_phase2"],
                      "frac_of_peak": (3.0 if p == "bf16x3" else 1.0) * v["gflops"] / 1e3 /
                      PEAK_TFLOPS["bf16" if p == "bf16x3" else p]}
                  for p, v in applies.items()},
        "roofline": roofline,
        "plan": tune,
        "setup_s": {"mpo": t_ham, "environments": t_env},
    }
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
