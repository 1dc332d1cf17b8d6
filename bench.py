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


def shift_for(spec, env, name, starts: int = 2):
    """E0 below the lowest eigenvalue of H_eff, so that Q(H_eff - E0)Q is positive definite.

    Lattice models (one-body + non-negative on-site U): E(U=0) - 0.5, a rigorous bound.  Ab initio:
    a heuristic -- the lowest Ritz value of 60-step Lanczos runs from two independent start
    vectors, minus max(0.5, 2 ||r||); the two Ritz values must agree within their residuals (a run
    that converged to a higher eigenvalue would show up as a disagreement), else the rule fails."""
    from workloads import configs as C
    if spec["eri"] is None:
        return C.lower_bound_shift(spec, 0.5), "E(U=0) - 0.5"
    t1, r1 = env.lowest_eigenvalue(steps=60, seed=7)
    if starts < 2:
        return t1 - max(0.5, 2.0 * r1), f"lanczos theta={t1:.12f} res={r1:.3e}, minus max(0.5, 2 res)"
    t2, r2 = env.lowest_eigenvalue(steps=60, seed=8)
    if abs(t1 - t2) > 2.0 * (r1 + r2) + 1e-9:
        raise RuntimeError(f"Lanczos runs disagree: {t1} (res {r1}) vs {t2} (res {r2})")
    res = max(r1, r2)
    return min(t1, t2) - max(0.5, 2.0 * res), (f"lanczos theta={t1:.12f}/{t2:.12f} res={r1:.3e}/{r2:.3e}, "
                                               f"minus max(0.5, 2 res)")


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
             (64, 128): (2, 2), (32, 64): (2, 2), (64, 32): (2, 2), (128, 128): (4, 2)}[(bm, bn)]
    kind = "packed" if launch.get("packed") else "terms"
    if precision == "bf16x3":
        if (bm, bn) == (128, 128):
            waves = (2, 2)  # the BF16x3 launcher runs this tile as four waves of 64x64
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


def _counter_rows(root: str, counter: str) -> list:
    """(kernel name, workgroups, value) of every dispatch in the rocprofv3 counter CSVs under root."""
    import csv
    import glob
    rows = []
    for path in glob.glob(os.path.join(root, "**", "*counter_collection.csv"), recursive=True):
        with open(path) as fh:
            for r in csv.DictReader(fh):
                if r.get("Counter_Name") != counter:
                    continue
                wg = int(r.get("Workgroup_Size") or 1)
                rows.append((r["Kernel_Name"], int(r["Grid_Size"]) // max(wg, 1), float(r["Counter_Value"])))
    return rows


def write_pmc_summary(fetch_dir: str, write_dir: str, workload: str, commands: list) -> dict:
    """profiles/pmc_traffic_<workload>.txt from two rocprofv3 --pmc runs of `--apply-only`
    (FETCH_SIZE, then WRITE_SIZE; KiB per dispatch): per kernel and workgroup count, the mean of
    each counter and the HBM bytes they stand for, scaled by what the same counter reads for the
    run's device copy of known size (256 MiB read and written)."""
    import re
    copy_bytes = 256.0 * 1024 * 1024
    out = {"workload": workload, "source_sha1": source_digest(), "commands": commands, "kernels": {}}
    means = {}
    for key, root, counter in (("fetch", fetch_dir, "FETCH_SIZE"), ("write", write_dir, "WRITE_SIZE")):
        per = {}
        copy = 0.0
        for name, wgs, val in _counter_rows(root, counter):
            if "copy" in name.lower():
                copy = max(copy, val)
                continue
            m = re.search(r"(gemm_\w+_kernel<[^>]*>|reduce_kernel<\w+>)", name)
            if not m:
                continue
            per.setdefault(f"{m.group(1)} x{wgs}", []).append(val)
        if copy <= 0:
            raise RuntimeError(f"no copy dispatch in {root}: the calibration needs it")
        out.setdefault("copy_kib", {})[key] = copy
        out.setdefault("scale", {})[key] = copy_bytes / (copy * 1024.0)
        means[key] = {k: (len(v), sum(v) / len(v)) for k, v in per.items()}
    for k in sorted(set(means["fetch"]) & set(means["write"])):
        n, f = means["fetch"][k]
        _, w = means["write"][k]
        out["kernels"][k] = {"dispatches": n, "fetch_kib": f, "write_kib": w,
                             "traffic_bytes": f * 1024.0 * out["scale"]["fetch"] + w * 1024.0 * out["scale"]["write"]}
    path = os.path.join(ROOT, "profiles", f"pmc_traffic_{workload}.txt")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")
    return out


def cpu_baseline_worker(workload: str, target_s: float) -> None:
    """Child process (CPU only, no GPU): the oracle's full-size contraction of the benchmarked
    workload (its own two-sided MPO, channel-stacked environments, the middle-bond
    factorisation) timed on whole H_eff x products until `target_s` seconds have run.  Prints one
    JSON line."""
    from oracle import mpo as OM
    from oracle import stacked as ST
    from workloads import configs as C
    from workloads import mps as M
    import threadpoolctl
    t0 = time.perf_counter()
    with threadpoolctl.threadpool_limits(limits=max(1, (os.cpu_count() or 2) // 2)):
        spec, mps = C.make(workload)
        fe = ST.FullSizeEnvironments(spec, mps, OM.build_mpo_twosided(spec))
    t_setup = time.perf_counter() - t0
    X = fe.to_sectors(M.random_two_site_vector(mps, 17))
    # the timed products start when the parent has finished its own work and waits
    print("ready", flush=True)
    sys.stdin.readline()
    reps, t_apply, flops = 0, 0.0, 0
    while t_apply < target_s and reps < 10:
        cnt = {}
        t0 = time.perf_counter()
        fe.apply_sectors(X, counter=cnt)
        t_apply += time.perf_counter() - t0
        flops += cnt["flops"]
        reps += 1
    blas = [{k: i.get(k) for k in ("internal_api", "num_threads", "version")} for i in threadpoolctl.threadpool_info()]
    threads = max([b.get("num_threads") or 1 for b in blas] or [1])
    print(json.dumps({"value": flops / t_apply / 1e9, "unit": "GFLOP/s", "cores": threads, "kind": "oracle",
                      "sample": (f"{reps} whole H_eff x product(s) of {workload} by the oracle (numpy FP64, "
                                 f"own two-sided MPO, D_mid = {len(fe.dq)}) in {t_apply:.1f} s after "
                                 f"{t_setup:.1f} s of untimed setup (MPO, environments, enlarged operators); "
                                 f"work = the {flops / reps:.4e} flops the oracle's products perform per apply"),
                      "blas": blas, "setup_s": t_setup}), flush=True)


def start_cpu_baseline(workload: str, target_s: float = 20.0):
    """Start the oracle's timing in a child process so that it runs beside the GPU measurements."""
    import subprocess
    return subprocess.Popen([sys.executable, os.path.abspath(__file__), "--cpu-baseline-worker", "--workload", workload,
                             "--cpu-baseline-seconds", str(target_s)], stdin=subprocess.PIPE, stdout=subprocess.PIPE,
                            stderr=subprocess.PIPE, text=True)


def finish_cpu_baseline(proc, timeout_s: float = 600.0):
    """Let the child start its timed products (the GPU work is over) and collect its line."""
    try:
        out, err = proc.communicate(input="go\n", timeout=timeout_s)
    except Exception as e:  # noqa: BLE001
        proc.kill()
        return {"value": None, "unit": "GFLOP/s", "cores": None, "kind": "oracle", "sample": f"oracle run failed: {e}"}
    for line in reversed(out.strip().splitlines()):
        try:
            return json.loads(line)
        except Exception:
            continue
    return {"value": None, "unit": "GFLOP/s", "cores": None, "kind": "oracle",
            "sample": "oracle run failed: " + err.strip().splitlines()[-1] if err.strip() else "no output"}


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
    print(json.dumps(measure_batch(args)), flush=True)


def measure_batch(args) -> dict:
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
    t_inputs = t_env = t_shift = 0.0
    for i, (parent, m, seed) in enumerate(members):
        ta = time.perf_counter()
        spec, mps = C.make_member(parent, m, seed)
        b_host = M.random_two_site_vector(mps, seed + 7)
        tb = time.perf_counter()
        if parent not in hams:
            hams[parent] = ctx.create_hamiltonian(spec)
        env = ctx.build_environments(hams[parent], mps)
        tc = time.perf_counter()
        e0, _ = shift_for(spec, env, parent, starts=1)
        td = time.perf_counter()
        t_inputs += tb - ta
        t_env += tc - tb
        t_shift += td - tc
        envs.append(env)
        e0s.append(e0)
        flops.append(env.flops_per_apply)
        bs.append(torch.tensor(env.pack(b_host), dtype=torch.float64, device=dev))
        log(f"[batch] member {i}: {parent} M={m} n={env.n} F={env.flops_per_apply:.3e} E0={e0:.6f} "
            f"(inputs {tb - ta:.1f}s, environments {tc - tb:.1f}s, shift {td - tc:.1f}s)")
    t_setup = time.perf_counter() - t0
    xs = [torch.zeros_like(b) for b in bs]
    batch = lcc.Batch(ctx, envs)
    status, infos = batch.solve(bs, e0s, xs, precision=args.precision, tol=1e-10, max_iter=5000,
                                inner_tol=args.inner_tol)  # warm-up
    torch.cuda.synchronize()
    reps = max(1, args.steps) if args.mode == "batch" else 1  # one timed batch inside the default line
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
           "setup_s": t_setup, "setup_split_s": {"inputs": t_inputs, "environments": t_env, "shift": t_shift},
           "intermediate_limit_mib": args.batch_intermediate_mib,
           "members": [{"parent": p, "m": m} for p, m, _ in members]}
    batch.close()
    for env in envs:
        env.close()
    return out


def measure_lattice(args, name: str) -> dict:
    """Apply throughput per precision and the local solve, mixed against FP64, on a lattice
    workload (E0 = E(U=0) - 0.5, a rigorous lower bound for these Hamiltonians)."""
    import torch
    from paper_1509_00216_amd import lcc
    from workloads import configs as C
    from workloads import mps as M
    dev = torch.device("cuda:0")
    spec, mps = C.make(name)
    ctx = lcc.Context(0)
    if not args.no_tune:
        ctx.set_tune_cache(working_tune_cache(args.tune_cache))
    env = ctx.build_environments(ctx.create_hamiltonian(spec), mps)
    F = env.flops_per_apply
    x64 = torch.tensor(env.pack(M.random_two_site_vector(mps, 17)), dtype=torch.float64, device=dev)
    out = {"vector_elements": env.n, "mpo_bond_dim_mid": env.mpo_bond_dim, "flops_per_apply": F, "apply": {}}
    for prec in ("fp64", "fp32", "bf16x3"):
        xx = x64 if prec == "fp64" else x64.float()
        yy = torch.empty_like(xx)
        env.apply_heff(xx, yy, prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.apply_reps):
            env.apply_heff(xx, yy, prec)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / args.apply_reps
        out["apply"][prec] = {"ms": ms, "gflops": F / (ms * 1e-3) / 1e9,
                              "frac_of_peak": (3.0 if prec == "bf16x3" else 1.0) * F / (ms * 1e-3) / 1e12 /
                              PEAK_TFLOPS["bf16" if prec == "bf16x3" else prec]}
    e0 = C.lower_bound_shift(spec, 0.5)
    b = torch.tensor(env.pack(M.random_two_site_vector(mps, 2025)), dtype=torch.float64, device=dev)
    x = torch.zeros_like(b)
    res = {}
    for prec in (args.precision, "fp64", args.precision, "fp64"):  # second pass timed
        x.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = env.solve_local_lcc(b, e0, x, precision=prec, tol=1e-10, max_iter=5000, inner_tol=args.inner_tol,
                                   max_outer=200)
        torch.cuda.synchronize()
        res[prec] = dict(info, ms=(time.perf_counter() - t0) * 1e3)
    out["solve"] = {"e0": e0, "mixed_precision": args.precision, "mixed_ms": res[args.precision]["ms"],
                    "fp64_ms": res["fp64"]["ms"], "speedup": res["fp64"]["ms"] / res[args.precision]["ms"],
                    "energy_diff": abs(res[args.precision]["hylleraas"] - res["fp64"]["hylleraas"]),
                    "hylleraas": res["fp64"]["hylleraas"],
                    "mixed_applies": [res[args.precision]["applies_low"], res[args.precision]["applies_fp64"]],
                    "fp64_applies": res["fp64"]["applies_fp64"]}
    env.close()
    return out


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



def run_small(args):
    """Local solves at a reduced bond dimension (--m-max) of --workload, where the small
    launches of the CG iteration weigh most: FP64 and mixed solves (one warm-up each, then
    --steps timed), with the operator product timed alone for comparison."""
    import torch
    from paper_1509_00216_amd import lcc
    from workloads import configs as C
    from workloads import mps as M
    torch.cuda.init()
    dev = torch.device("cuda:0")
    spec, mps = C.make(args.workload, m_max=args.m_max)
    ctx = lcc.Context(0)
    ctx.set_tune_cache(working_tune_cache(args.tune_cache))
    env = ctx.build_environments(ctx.create_hamiltonian(spec), mps)
    e0, rule = shift_for(spec, env, args.workload)
    b = torch.tensor(env.pack(M.random_two_site_vector(mps, 2025)), dtype=torch.float64, device=dev)
    x = torch.zeros_like(b)
    out = {"mode": "small", "workload": args.workload, "m_max": args.m_max, "n": env.n, "e0_rule": rule}
    for prec in ("fp64", args.precision):
        xx = b if prec == "fp64" else b.float()
        yy = torch.empty_like(xx)
        env.apply_heff(xx, yy, prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(20):
            env.apply_heff(xx, yy, prec)
        torch.cuda.synchronize()
        ms_apply = (time.perf_counter() - t0) * 1e3 / 20
        times, info = [], None
        for rep in range(1 + max(1, args.steps)):
            x.zero_()
            torch.cuda.synchronize()
            time.sleep(0.05)  # idle gap: the solves stand apart in a kernel trace
            t0 = time.perf_counter()
            info = env.solve_local_lcc(b, e0, x, precision=prec, tol=1e-10, max_iter=5000, inner_tol=args.inner_tol,
                                       max_outer=200)
            torch.cuda.synchronize()
            if rep > 0:
                times.append((time.perf_counter() - t0) * 1e3)
        out[prec] = {"ms_apply": ms_apply, "ms_solve": sum(times) / len(times), "iterations": info["iterations"],
                     "applies_fp64": info["applies_fp64"], "applies_low": info["applies_low"],
                     "J": info["hylleraas"], "rel_residual": info["rel_residual"]}
        log(f"[small] {prec}: {out[prec]}")
    env.close()
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
    ap.add_argument("--mode", default="solve", choices=["solve", "batch", "sweep", "tune", "small"],
                    help="solve: the headline local solve (default); batch: 64 independent problems, batched "
                         "mixed vs sequential FP64; sweep: one sweep of the 4x4 Hubbard model; tune: autotune "
                         "--tune-workloads into --tune-cache; small: local solves of --workload at bond "
                         "dimension --m-max")
    ap.add_argument("--m-max", type=int, default=128, help="bond dimension of --mode small")
    ap.add_argument("--tune-cache", default=SHIPPED_TUNE_CACHE)
    ap.add_argument("--tune-workloads", default="abinitio_k24_m1000,threeband_4x2_m2000,hubbard2d_4x4_m500")
    ap.add_argument("--no-tune", action="store_true", help="plan with the default planner parameters")
    ap.add_argument("--inner-tol", type=float, default=1e-5,
                    help="mixed precision: residual reduction between FP64 refreshes (1e-5: two refreshes "
                         "to 1e-10 at K=24, M=1000; 1e-4 needs three, 3e-6 more FP32 iterations)")
    ap.add_argument("--batch-n", type=int, default=64)
    ap.add_argument("--batch-intermediate-mib", type=int, default=1024)
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the extra keys (3-band M=2000 cluster; 64 batched problems)")
    ap.add_argument("--cpu-baseline-seconds", type=float, default=20.0)
    ap.add_argument("--cpu-baseline-worker", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--pmc-summary", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="write profiles/pmc_traffic_<workload>.txt from the rocprofv3 counter output of two "
                         "--apply-only runs (FETCH_SIZE, WRITE_SIZE); no GPU needed")
    args = ap.parse_args()
    if args.cpu_baseline_worker:
        return cpu_baseline_worker(args.workload, args.cpu_baseline_seconds)
    if args.pmc_summary:
        cmd = ("cd /tmp && export TMPDIR=/tmp && timeout -s KILL 150 rocprofv3 --pmc {c} --output-format csv -d "
               "<out>/{d} -o apply -- python3 $R/bench.py --workload %s --apply-only 3 --apply-precision fp32"
               % args.workload)
        rec = write_pmc_summary(args.pmc_summary[0], args.pmc_summary[1], args.workload,
                                [cmd.format(c="FETCH_SIZE", d="fetch"), cmd.format(c="WRITE_SIZE", d="write")])
        print(json.dumps({"mode": "pmc-summary", "kernels": len(rec["kernels"]), "scale": rec["scale"]}))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (--gpus must be 1)", file=sys.stderr)
        sys.exit(2)

    if args.mode == "tune":
        return run_tune(args)
    if args.mode == "batch":
        return run_batch(args)
    if args.mode == "sweep":
        return run_sweep(args)
    if args.mode == "small":
        return run_small(args)

    # the oracle's timing runs in a child process on the host cores beside the GPU measurements
    baseline = None
    if not args.no_cpu_baseline and args.apply_only <= 0:
        baseline = start_cpu_baseline(args.workload, args.cpu_baseline_seconds)

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
    log(f"[bench] environments in {t_env:.2f}s: n={env.n} D_mid={env.mpo_bond_dim} F_alg={F:.4e} (left operator {f1:.3e}, right operator {f2:.3e})")
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
                          "ms_per_apply": ms, "flops_per_apply": F, "left_flops": f1, "right_flops": f2,
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
    other = None
    if args.precision == "fp32":
        # the same mixed solve with the BF16x3 split-product operator inside the refinement
        t0 = time.perf_counter()
        info_bf = solve("bf16x3")
        torch.cuda.synchronize()
        other = {"ms": (time.perf_counter() - t0) * 1e3, "applies_low": info_bf["applies_low"],
                 "applies_fp64": info_bf["applies_fp64"], "hylleraas": info_bf["hylleraas"],
                 "energy_diff_vs_fp32": abs(info_bf["hylleraas"] - j_mixed), "status": info_bf["status"]}
        log(f"[bench] bf16x3 mixed solve: {info_bf}")

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
                  "fp64": fp64, "bf16x3": other,
                  "energy_diff_vs_fp64": (abs(j_mixed - fp64["hylleraas"]) if fp64 else None),
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
    env.close()
    if not args.no_extra:
        log("[bench] 3-band cluster, M=2000")
        out["threeband_4x2_m2000"] = measure_lattice(args, "threeband_4x2_m2000")
        log(f"[bench] {out['threeband_4x2_m2000']}")
        log(f"[bench] {args.batch_n} batched problems")
        out["batch64"] = measure_batch(args)
        log(f"[bench] batch: {out['batch64']['ms_batched_mixed']:.0f} ms batched vs "
            f"{out['batch64']['ms_sequential_fp64']:.0f} ms sequential FP64")
    if baseline is not None:
        log("[bench] waiting for the oracle's timing (cpu baseline)")
        out["cpu_baseline"] = finish_cpu_baseline(baseline)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
