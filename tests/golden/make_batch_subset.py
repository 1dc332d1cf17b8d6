"""Writes batch_subset.json: oracle energies of the first eight lattice members (4x4 Hubbard and
3-band parents) of the seeded 64-problem batch, at their full bond dimensions (M between
362 and 1469).

Calls only oracle/ and the input generators of workloads/.  For each member: the parent's
Hamiltonian, the member's jittered random MPS, E0 = E(U=0) - 0.5 (a rigorous lower bound for
these Hamiltonians), b = the seeded unit vector of seed (member seed + 7), and x* of
(H_eff - E0) x = b by plain CG to a relative residual of 1e-12 on the oracle's full-size
contraction; J* = -b^T x*.

Run: python tests/golden/make_batch_subset.py
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

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "batch_subset.json")


def main():
    members = [(i, p, m, s) for i, (p, m, s) in enumerate(C.batch_members(64)) if p != "abinitio_k24_m1000"][:8]
    out = []
    for i, parent, m, seed in members:
        t0 = time.time()
        spec, mps = C.make_member(parent, m, seed)
        fe = ST.FullSizeEnvironments(spec, mps, OM.build_mpo(spec))
        blocks = M.two_site_blocks(mps)
        tmpl = BS.two_site_template(mps, blocks)
        n = sum(v.size for v in tmpl.values())
        ap = lambda z: BS.flatten(fe.apply(BS.unflatten(z, tmpl, blocks)), blocks)
        e0 = C.lower_bound_shift(spec, 0.5)
        b = BS.flatten(M.random_two_site_vector(mps, seed + 7), blocks)
        xs, it, rel, _ = OS.cg(OS.make_operator(ap, e0), b, tol=1e-12, max_iter=4000)
        rec = {"index": i, "parent": parent, "m": m, "seed": seed, "n": int(n), "e0": e0, "b_seed": seed + 7,
               "iterations": it, "rel_residual": rel, "hylleraas": float(-(b @ xs))}
        out.append(rec)
        print(f"member {i} {parent} M={m} n={n}: J* {rec['hylleraas']:.15f} ({it} it, {time.time() - t0:.0f} s)",
              flush=True)
    with open(OUT, "w") as f:
        json.dump({"members": out}, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
