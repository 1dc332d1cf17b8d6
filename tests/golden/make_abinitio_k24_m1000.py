"""Writes abinitio_k24_m1000.json: oracle results for the benchmarked ab initio workload
(24 orbitals, 12 electrons, 2Sz = 0, bond dimension 1000, two-site block at the chain centre).

Calls only oracle/ (the two-sided MPO and the full-size block-sparse contraction) and the input
generators of workloads/; nothing here comes from the library under test.

* apply: y = H_eff x for the seeded unit vector x (seed 5): sampled entries of y (2048 elements
  drawn uniformly, seeded), ||y|| and <z, y> for a second seeded vector z (seed 6).
* shift: the lowest Ritz value theta of a 60-step Lanczos on H_eff and its residual, and
  E0 = theta - max(0.5, 2 ||r||) (the shift rule used for this workload).
* solve: x* of (H_eff - E0) x = b for the seeded b (seed 2025) by plain CG to a relative
  residual of 1e-12; the Hylleraas value J* = -b^T x* and 2048 sampled entries of x*.

Run: python tests/golden/make_abinitio_k24_m1000.py   (about an hour on 8 cores)
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import blocksparse as BS  # noqa: E402
from oracle import mpo as OM  # noqa: E402
from oracle import solve as OS  # noqa: E402
from oracle import stacked as ST  # noqa: E402
from workloads import configs as C  # noqa: E402
from workloads import mps as M  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "abinitio_k24_m1000.json")


def log(msg):
    print(f"[{time.strftime('%H:%M:%S')}] {msg}", flush=True)


def samples(vec_flat, blocks, tmpl, count, seed):
    """`count` entries drawn uniformly over all elements: [ia, s1, s2, ib, i, j, value]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    starts, off = [], 0
    for k in blocks:
        starts.append(off)
        off += tmpl[k].size
    picks = np.sort(rng.choice(off, size=count, replace=False))
    out = []
    bi = 0
    for p in picks:
        while bi + 1 < len(starts) and starts[bi + 1] <= p:
            bi += 1
        k = blocks[bi]
        i, j = divmod(int(p - starts[bi]), tmpl[k].shape[1])
        out.append([int(k[0]), int(k[1]), int(k[2]), int(k[3]), i, j, float(vec_flat[p])])
    return out


def main():
    spec, mps = C.make("abinitio_k24_m1000")
    log("oracle MPO")
    mpo = OM.build_mpo_twosided(spec)
    log("environments and enlarged operators")
    fe = ST.FullSizeEnvironments(spec, mps, mpo)
    blocks = M.two_site_blocks(mps)
    tmpl = BS.two_site_template(mps, blocks)
    n = sum(v.size for v in tmpl.values())

    def ap(z):
        return BS.flatten(fe.apply(BS.unflatten(z, tmpl, blocks)), blocks)

    out = {"workload": "abinitio_k24_m1000", "n": int(n), "oracle_mpo_bond_dim_mid": len(mpo["dq"][mps["center"] + 1])}
    x = BS.flatten(M.random_two_site_vector(mps, 5), blocks)
    z = BS.flatten(M.random_two_site_vector(mps, 6), blocks)
    log("apply")
    y = ap(x)
    out["apply"] = {"x_seed": 5, "z_seed": 6, "norm_y": float(np.linalg.norm(y)), "z_dot_y": float(z @ y),
                    "samples": samples(y, blocks, tmpl, 2048, 11)}
    log("lanczos")
    th, res, _ = OS.lanczos_lowest(ap, n, steps=60, seed=0)
    e0 = th - max(0.5, 2.0 * res)
    out["shift"] = {"lanczos_steps": 60, "lanczos_seed": 0, "theta": th, "residual": res, "e0": e0}
    log(f"theta {th:.12f} res {res:.3e} e0 {e0:.12f}; CG")
    b = BS.flatten(M.random_two_site_vector(mps, 2025), blocks)
    A = OS.make_operator(ap, e0)
    xs, it, rel, hist = OS.cg(A, b, tol=1e-12, max_iter=2000)
    jstar = float(-(b @ xs))
    log(f"CG {it} iterations, rel residual {rel:.3e}, J* {jstar:.15f}, last J(x_k) {hist[-1]:.15f}")
    out["solve"] = {"b_seed": 2025, "tol": 1e-12, "iterations": it, "rel_residual": rel, "hylleraas": jstar,
                    "hylleraas_recurrence": hist[-1], "samples_x": samples(xs, blocks, tmpl, 2048, 12)}
    with open(OUT, "w") as f:
        json.dump(out, f)
        f.write("\n")
    log(f"wrote {OUT}")


if __name__ == "__main__":
    main()
