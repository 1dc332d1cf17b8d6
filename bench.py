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
    for f in ("kernels.hip", "env.cpp", "internal.h"):
        with open(os.path.join(ROOT, "paper_1509_00216_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def kernel_name(precision: str, launch: dict) -> str:
    if launch["kind"] == "reduce":
        return "reduce_kernel<%s>" % ("double" if precision == "fp64" else "float")
    tb = "true" if launch["phase"] == 2 else "false"
    bm, bn = launch["tile"]
    waves = {(64, 64): (2, 2), (16, 64): (1, 4), (64, 16): (4, 1), (32, 32): (2, 2), (128, 64): (2, 2),
             (64, 128): (2, 2), (32, 64): (2, 2), (64, 32): (2, 2)}[(bm, bn)]
    if precision == "bf16x3":
        return f"gemm_bf16x3_kernel<false, {tb}, {bm}, {bn}, {waves[0]}, {waves[1]}>"
    mode = 0 if precision == "fp64" else 1
    return f"gemm_mfma_kernel<{mode}, false, {tb}, {bm}, {bn}, {waves[0]}, {waves[1]}>"


def measured_traffic(kname: str, workload: str):
    """HBM bytes per launch of `kname` from the committed PMC summary, if the kernel sources
    have not changed since the counters were taken (else None)."""
    path = os.path.join(ROOT, "profiles", f"pmc_traffic_{workload}.txt")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
    except Exception:
        return None
    if rec.get("source_sha1") != source_digest():
        return None
    ent = rec.get("kernels", {}).get(kname)
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
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (--gpus must be 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1509_00216_amd import lcc
    from workloads import configs as C
    from workloads import mps as M

    torch.cuda.init()
    dev = torch.device("cuda:0")
    log(f"[bench] workload {args.workload}: generating inputs")
    spec, mps = C.make(args.workload)
    ctx = lcc.Context(0)
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
        applies[prec] = {"ms_phase1": ms1, "ms_phase2": ms2, "ms": ms1 + ms2,
                         "gflops": F / ((ms1 + ms2) * 1e-3) / 1e9}
        log(f"[bench] apply {prec}: phase1 {ms1:.3f} ms, phase2 {ms2:.3f} ms, {applies[prec]['gflops']:.1f} GFLOP/s")

    # --- timed steps: mixed-precision local solves from x = 0
    b = torch.tensor(env.pack(M.random_two_site_vector(mps, 2025)), dtype=torch.float64, device=dev)
    x = torch.zeros_like(b)

    def solve(prec):
        x.zero_()
        return env.solve_local_lcc(b, e0, x, precision=prec, tol=1e-10, max_iter=5000)

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
                "traffic": measured_traffic(kname, args.workload), "kernel": kname,
                "launch_ms": dom["ms"], "launch_flops": dom["flops"], "launch_algorithmic_bytes": dom["bytes"],
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
        "solve": {"precision": args.precision, "ms": ms_step, "iterations": infos[-1]["iterations"],
                  "outer": infos[-1]["outer"], "applies_fp64": infos[-1]["applies_fp64"],
                  "applies_low": infos[-1]["applies_low"], "hylleraas": j_mixed,
                  "rel_residual": infos[-1]["rel_residual"], "e0": e0,
                  "fp64": fp64, "energy_diff_vs_fp64": (abs(j_mixed - fp64["hylleraas"]) if fp64 else None),
                  "speedup_vs_fp64": (fp64["ms"] / ms_step if fp64 else None)},
        "apply": {p: {"gflops": v["gflops"], "ms": v["ms"], "ms_phase1": v["ms_phase1"], "ms_phase2": v["ms_phase2"],
                      "frac_of_peak": (3.0 if p == "bf16x3" else 1.0) * v["gflops"] / 1e3 /
                      PEAK_TFLOPS["bf16" if p == "bf16x3" else p]}
                  for p, v in applies.items()},
        "roofline": roofline,
        "setup_s": {"mpo": t_ham, "environments": t_env},
    }
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
