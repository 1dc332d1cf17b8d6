"""Oracle of one left-to-right sweep of two-site local solves (Implementation section: the
tensors are optimised one at a time, sweeping over the sites), plain numpy FP64.

At each block the local problem Q(H_eff - e0)Q x = Q b is solved by plain CG; x is split per
middle-bond sector with numpy's SVD, the m_max largest singular values over all sectors are
kept (ties: sector (N, 2Sz) ascending, then index), U becomes the left-canonical tensor of the
left site, and S V^T contracted with the next site's right-canonical tensor is the next
block's guess.  Environments are recomputed from scratch with oracle.blocksparse at every
block.  Only gauge-invariant quantities (energies, singular values) are comparable with
another implementation, because singular vectors carry a free sign per vector.
"""
from __future__ import annotations

import numpy as np

SV_CUT = 1e-10  # singular values below SV_CUT * the largest are treated as zero

from . import blocksparse as BS
from . import solve as OS
from .mpo import LOCAL_QN


def _sectors_of_block(mps: dict, l: int):
    bl, br = mps["bonds"][l], mps["bonds"][l + 2]
    mid = {}
    for ia, (n, z, d) in enumerate(bl):
        for s1, (dn, dz) in enumerate(LOCAL_QN):
            mid.setdefault((n + dn, z + dz), {"rows": [], "cols": []})["rows"].append((ia, s1))
    for ib, (n, z, d) in enumerate(br):
        for s2, (dn, dz) in enumerate(LOCAL_QN):
            key = (n - dn, z - dz)
            if key in mid:
                mid[key]["cols"].append((s2, ib))
    return {q: v for q, v in sorted(mid.items()) if v["rows"] and v["cols"]}


def split(x: dict, mps: dict, m_max: int):
    """Return (new site-l blocks, new bond l+1, guess for block l+1 as a dict, all singular values)."""
    l = mps["center"]
    bl, br = mps["bonds"][l], mps["bonds"][l + 2]
    secs = _sectors_of_block(mps, l)
    svd = {}
    cand = []
    for qi, (q, S) in enumerate(secs.items()):
        rows = [bl[ia][2] for ia, _ in S["rows"]]
        cols = [br[ib][2] for _, ib in S["cols"]]
        X = np.zeros((sum(rows), sum(cols)))
        r0 = 0
        for (ia, s1), nr in zip(S["rows"], rows):
            c0 = 0
            for (s2, ib), nc in zip(S["cols"], cols):
                blk = x.get((ia, s1, s2, ib))
                if blk is not None:
                    X[r0:r0 + nr, c0:c0 + nc] = blk
                c0 += nc
            r0 += nr
        U, s, Vt = np.linalg.svd(X, full_matrices=False)
        svd[q] = (U, s, Vt, rows, cols)
        cand.extend((float(v), qi, i, q) for i, v in enumerate(s))
    cand.sort(key=lambda c: (-c[0], c[1], c[2]))
    keep = {}
    # singular values at the rounding level of the largest are zeros of the exact tensor: their
    # vectors are not determined, so they are never kept (reading: relative cut 1e-10)
    cut = SV_CUT * (cand[0][0] if cand else 0.0)
    for c in cand[:m_max]:
        if c[0] > cut:
            keep[c[3]] = max(keep.get(c[3], 0), c[2] + 1)
    new_bond = [(q[0], q[1], keep[q]) for q in secs if q in keep]
    new_index = {q: i for i, (q0, q1, _) in enumerate(new_bond) for q in [(q0, q1)]}
    site_blocks = []
    for q, S in secs.items():
        if q not in keep:
            continue
        U = svd[q][0]
        r0 = 0
        for (ia, s1), nr in zip(S["rows"], svd[q][3]):
            site_blocks.append((ia, s1, new_index[q], U[r0:r0 + nr, :keep[q]].copy()))
            r0 += nr
    # guess: (S V^T)_q [:, (s2, b)] B_{l+2}^{s3}[b -> c]  ->  keys (iq, s2, s3, ic) of block l+1
    Bsite = {(il, s): (ir, a) for il, s, ir, a in mps["sites"][l + 2]}
    guess = {}
    for q, S in secs.items():
        if q not in keep:
            continue
        _, s, Vt, _, cols = svd[q]
        C = s[:keep[q], None] * Vt[:keep[q], :]
        c0 = 0
        for (s2, ib), nc in zip(S["cols"], cols):
            part = C[:, c0:c0 + nc]
            c0 += nc
            for s3 in range(4):
                hit = Bsite.get((ib, s3))
                if hit is None:
                    continue
                ic, B = hit
                key = (new_index[q], s2, s3, ic)
                guess[key] = guess.get(key, 0.0) + part @ B
    return site_blocks, new_bond, guess, np.array(sorted((c[0] for c in cand), reverse=True))


def advance(mps: dict, site_blocks, new_bond) -> dict:
    """The MPS with site l replaced and bond l+1 truncated; the block moves to l+1."""
    l = mps["center"]
    bonds = list(mps["bonds"])
    bonds[l + 1] = new_bond
    sites = list(mps["sites"])
    sites[l] = site_blocks
    return dict(mps, bonds=bonds, sites=sites, center=l + 1)


def local_solve(spec: dict, mps: dict, mpo: dict, b: dict, e0: float, tol: float = 1e-13):
    """x* and J* of the local problem at the block mps['center'] (no projector)."""
    env = BS.Environments(spec, mps, mpo)
    from workloads import mps as M  # block enumeration of the generator (inputs only)
    blocks = M.two_site_blocks(mps)
    tmpl = BS.two_site_template(mps, blocks)
    bfull = {k: b.get(k, np.zeros_like(v)) for k, v in tmpl.items()}
    ap = lambda z: BS.flatten(env.apply(BS.unflatten(z, tmpl, blocks)), blocks)
    A = OS.make_operator(ap, e0)
    bf = BS.flatten(bfull, blocks)
    x, it, rel, _ = OS.cg(A, bf, tol=tol, max_iter=5000)
    return BS.unflatten(x, tmpl, blocks), OS.hylleraas(A, x, bf), it


def local_ground_state(spec: dict, mps: dict, mpo: dict):
    """Lowest eigenpair (theta, u as a block dict) of H_eff at the block mps['center'].

    The DMRG energy functional of the Implementation section is stationary where H_eff u =
    theta u; the local step of a ground-state sweep takes the lowest such pair.  H_eff is formed
    densely here, column by column from oracle.blocksparse, and diagonalised with numpy (small
    blocks only)."""
    env = BS.Environments(spec, mps, mpo)
    from workloads import mps as M  # block enumeration of the generator (inputs only)
    blocks = M.two_site_blocks(mps)
    tmpl = BS.two_site_template(mps, blocks)
    n = sum(v.size for v in tmpl.values())
    heff = np.zeros((n, n))
    for c in range(n):
        e = np.zeros(n)
        e[c] = 1.0
        heff[:, c] = BS.flatten(env.apply(BS.unflatten(e, tmpl, blocks)), blocks)
    w, U = np.linalg.eigh(0.5 * (heff + heff.T))
    return float(w[0]), BS.unflatten(U[:, 0], tmpl, blocks), float(w[1] - w[0]) if n > 1 else np.inf
