"""Exact algorithmic flop counts of one two-site H_eff x, from the block tables alone.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The Implementation section puts the cost of the H0 term of a sweep step at O(k^2 M^3): the
products of the left environment, the two MPO site tensors and the right environment with
the local tensor.  These functions count that work exactly, as integers, for a given MPS
block structure and a given MPO, without doing any arithmetic on tensor entries: a block
exists when the (N, 2Sz) selection rule and the MPO's nonzero pattern allow it, whatever
its values.  Two orders of the same contraction are counted:

canonical (L, then the MPO pair, then R), with W12^{w,w2} = sum_{w1} W_l^{w,w1} (x) W_{l+1}^{w1,w2}:
  K1  T_w[a', s1 s2 b]        = L^w[a' <- a] X[a, s1 s2 b]          2 M_a' M_a M_b per block pair
  K2  Z_w2[a', s1' s2', b]   += W12^{w,w2}[s1's2', s1s2] T_w[...]    2 M_a' M_b per entry and block
  K3  y[a', s1' s2', b']     += Z_w2[a', s1's2', b] R^{w2}[b' <- b]^T 2 M_a' M_b M_b'
  counting only T and Z blocks that reach an allowed y block.

factorised over the middle MPO bond (H_eff = sum_{w1} Lt^{w1} (x) Rt^{w1}, where Lt absorbs
W_l into L and Rt absorbs W_{l+1} into R), with the two-site vector stored per middle-bond
sector q as a matrix X_q (rows (a, s1), columns (s2, b)), in either order:
  left operator first
    T_{w1,q}  = Lt^{w1} X_q          2 M_a' M_a ncols(q) per nonzero block of Lt^{w1}
    Y_{q'}   += T_{w1,q} Rt^{w1 T}   2 nrows(q') M_b M_b' per nonzero block of Rt^{w1}
  right operator first
    T_{w1,q}  = X_q Rt^{w1 T}        2 nrows(q) M_b M_b' per nonzero block of Rt^{w1}
    Y_{q'}   += Lt^{w1} T_{w1,q}     2 M_a' M_a ncols(q') per nonzero block of Lt^{w1}
  for the (w1, q) pairs where both Lt^{w1} and Rt^{w1} read sector q and q' = q + dq(w1)
  is a sector of the block.  The counts are reported per operator ('left': products with Lt,
  'right': products with Rt), whichever runs first.

`mpo` is a dict in the oracle's format (oracle.mpo): per bond the channel shifts 'dq', per
site 'W' = {(w_in, w_out): 4x4 array}; any exact MPO of the Hamiltonian may be passed.
Whether a count is right is checked in the tests against the work that the oracle's own
contractions perform (counted multiply-adds) and against the M^3 scaling of the cost.
"""
from __future__ import annotations

from .mpo import LOCAL_QN


def _qn(bond, i):
    n, z, _ = bond[i]
    return (n, z)


def _sector_index(bond):
    return {(n, z): i for i, (n, z, _) in enumerate(bond)}


def left_structure(mps: dict, mpo: dict, upto: int) -> dict:
    """Blocks of the left environment at bond `upto`: {w: set of (row sector, column sector)}.

    Transition-element figure: L_{j+1}^{w'} collects A^{s'T} L_j^w A^s for every MPO entry
    (w, w') of site j with <s'|W|s> != 0 and every block of L_j^w whose sectors continue
    through site j in both the bra and the ket."""
    env = {0: {(0, 0)}}
    for j in range(upto):
        by_left = {}
        for il, s, ir, _ in mps["sites"][j]:
            by_left[(il, s)] = ir
        new = {}
        for (w, w2), m in mpo["W"][j].items():
            if w not in env:
                continue
            for (rp, r) in env[w]:
                for sp in range(4):
                    for s in range(4):
                        if m[sp, s] == 0.0:
                            continue
                        a = by_left.get((r, s))
                        ap = by_left.get((rp, sp))
                        if a is not None and ap is not None:
                            new.setdefault(w2, set()).add((ap, a))
        env = new
    return env


def right_structure(mps: dict, mpo: dict, fromsite: int) -> dict:
    """Blocks of the right environment at bond `fromsite`: {w: set of (row sector, column sector)}."""
    K = mps["n_sites"]
    env = {0: {(0, 0)}}
    for j in range(K - 1, fromsite - 1, -1):
        by_right = {}
        for il, s, ir, _ in mps["sites"][j]:
            by_right[(ir, s)] = il
        new = {}
        for (w, w2), m in mpo["W"][j].items():
            if w2 not in env:
                continue
            for (rp, r) in env[w2]:
                for sp in range(4):
                    for s in range(4):
                        if m[sp, s] == 0.0:
                            continue
                        b = by_right.get((r, s))
                        bp = by_right.get((rp, sp))
                        if b is not None and bp is not None:
                            new.setdefault(w, set()).add((bp, b))
        env = new
    return env


def _two_site_keys(mps):
    """Allowed blocks (a, s1, s2, b) of the two-site tensor (same rule as the input generator)."""
    l = mps["center"]
    bl, br = mps["bonds"][l], mps["bonds"][l + 2]
    rix = _sector_index(br)
    keys = set()
    for ia in range(len(bl)):
        n, z = _qn(bl, ia)
        for s1, (d1, z1) in enumerate(LOCAL_QN):
            for s2, (d2, z2) in enumerate(LOCAL_QN):
                ib = rix.get((n + d1 + d2, z + z1 + z2))
                if ib is not None:
                    keys.add((ia, s1, s2, ib))
    return keys


def canonical_flops(mps: dict, mpo: dict) -> dict:
    """Counts of the canonical order: {'k1', 'k2', 'k3', 'total'} (integers)."""
    l = mps["center"]
    dl = [d for _, _, d in mps["bonds"][l]]
    dr = [d for _, _, d in mps["bonds"][l + 2]]
    L = left_structure(mps, mpo, l)
    R = right_structure(mps, mpo, l + 2)
    ykeys = _two_site_keys(mps)
    # W12 pattern: (w, w2) -> set of ((s1', s2'), (s1, s2)) with a nonzero summed entry
    import numpy as np
    w12 = {}
    right = {}
    for (w1, w2), m2 in mpo["W"][l + 1].items():
        right.setdefault(w1, []).append((w2, m2))
    for (w, w1), m1 in mpo["W"][l].items():
        for w2, m2 in right.get(w1, []):
            w12[(w, w2)] = w12.get((w, w2), 0.0) + np.kron(m1, m2)
    pattern = {}
    for key, m in w12.items():
        nz = [((r // 4, r % 4), (c // 4, c % 4)) for r in range(16) for c in range(16) if m[r, c] != 0.0]
        if nz:
            pattern[key] = nz
    # Z blocks that reach an allowed y block: (w2, a', s1', s2', b)
    y_by_right = {}
    for (a, s1, s2, b) in ykeys:
        y_by_right.setdefault(b, []).append((a, s1, s2))
    z_used = {}
    for w2, blocks in R.items():
        for (bp, b) in blocks:
            for (ap, s1p, s2p) in y_by_right.get(bp, []):
                z_used.setdefault(w2, set()).add((ap, s1p, s2p, b))
    # T blocks that exist: (w, a', s1, s2, b) with L^w[a' <- a] and x[a, s1, s2, b]
    x_by_left = {}
    for (a, s1, s2, b) in ykeys:
        x_by_left.setdefault(a, []).append((s1, s2, b))
    t_exists = {}
    for w, blocks in L.items():
        for (ap, a) in blocks:
            for (s1, s2, b) in x_by_left.get(a, []):
                t_exists.setdefault(w, {})[(ap, s1, s2, b)] = a
    # K2 contributions and the T blocks they need
    k2 = 0
    t_used = set()
    z_made = set()
    for (w, w2), nz in pattern.items():
        tw = t_exists.get(w)
        zu = z_used.get(w2)
        if not tw or not zu:
            continue
        for (ap, s1, s2, b) in tw:
            for (s1p, s2p), (c1, c2) in nz:
                if (c1, c2) != (s1, s2):
                    continue
                if (ap, s1p, s2p, b) in zu:
                    k2 += 2 * dl[ap] * dr[b]
                    t_used.add((w, ap, s1, s2, b))
                    z_made.add((w2, ap, s1p, s2p, b))
    k1 = 0
    for (w, ap, s1, s2, b) in t_used:
        a = t_exists[w][(ap, s1, s2, b)]
        k1 += 2 * dl[ap] * dl[a] * dr[b]
    k3 = 0
    for (w2, ap, s1p, s2p, b) in z_made:
        for (bp, bb) in R[w2]:
            if bb == b and (ap, s1p, s2p, bp) in ykeys:
                k3 += 2 * dl[ap] * dr[b] * dr[bp]
    return {"k1": k1, "k2": k2, "k3": k3, "total": k1 + k2 + k3}


def middle_sectors(mps: dict, one_site: bool = False) -> list:
    """Middle-bond sectors q of the two-site block with their rows (a, s1) and columns (s2, b),
    in (N, 2Sz) order; rows by (a, s1), columns by (s2, b).  one_site: the site tensor at the
    center, rows (a, s1) and columns b of the next bond, written (0, b) (the empty local state,
    no charge)."""
    l = mps["center"]
    bl, br = mps["bonds"][l], mps["bonds"][l + (1 if one_site else 2)]
    rows, cols = {}, {}
    for ia in range(len(bl)):
        n, z = _qn(bl, ia)
        for s1, (d1, z1) in enumerate(LOCAL_QN):
            rows.setdefault((n + d1, z + z1), []).append((ia, s1))
    for s2, (d2, z2) in enumerate(LOCAL_QN[:1] if one_site else LOCAL_QN):
        for ib in range(len(br)):
            n, z = _qn(br, ib)
            cols.setdefault((n - d2, z - z2), []).append((s2, ib))
    out = []
    for q in sorted(rows):
        if q in cols:
            r = sorted(rows[q])
            c = sorted(cols[q])
            out.append({"q": q, "rows": r, "cols": c,
                        "nrows": sum(bl[a][2] for a, _ in r), "ncols": sum(br[b][2] for _, b in c)})
    return out


def enlarged_structure(mps: dict, mpo: dict, one_site: bool = False):
    """Nonzero blocks of the enlarged operators of the middle bond:
    lt[w1] = set of ((a', s1'), (a, s1)),  rt[w1] = set of ((s2', b'), (s2, b)),
    restricted to rows and columns of the block's middle sectors.  one_site: rt[w1] is the right
    environment R^{w1} of the sites right of the center itself, on columns (0, b)."""
    l = mps["center"]
    L = left_structure(mps, mpo, l)
    R = right_structure(mps, mpo, l + (1 if one_site else 2))
    secs = middle_sectors(mps, one_site)
    row_ok = {r for S in secs for r in S["rows"]}
    col_ok = {c for S in secs for c in S["cols"]}
    lt, rt = {}, {}
    for (w, w1), m in mpo["W"][l].items():
        for (ap, a) in L.get(w, ()):
            for sp in range(4):
                for s in range(4):
                    if m[sp, s] != 0.0 and (ap, sp) in row_ok and (a, s) in row_ok:
                        lt.setdefault(w1, set()).add(((ap, sp), (a, s)))
    if one_site:
        for w1, blocks in R.items():
            for (bp, b) in blocks:
                if (0, bp) in col_ok and (0, b) in col_ok:
                    rt.setdefault(w1, set()).add(((0, bp), (0, b)))
        return secs, lt, rt
    for (w1, w2), m in mpo["W"][l + 1].items():
        for (bp, b) in R.get(w2, ()):
            for sp in range(4):
                for s in range(4):
                    if m[sp, s] != 0.0 and (sp, bp) in col_ok and (s, b) in col_ok:
                        rt.setdefault(w1, set()).add(((sp, bp), (s, b)))
    return secs, lt, rt


def factorised_flops(mps: dict, mpo: dict, order: str = "left", one_site: bool = False) -> dict:
    """Counts of the middle-bond factorisation, {'left', 'right', 'total'} (integers), with the
    left (order "left") or the right (order "right") enlarged operator applied first; one_site:
    of the one-site problem at the center (right enlarged operator = R)."""
    if order not in ("left", "right"):
        raise ValueError(order)
    l = mps["center"]
    bl, br = mps["bonds"][l], mps["bonds"][l + (1 if one_site else 2)]
    secs, lt, rt = enlarged_structure(mps, mpo, one_site)
    sec_of_row = {r: i for i, S in enumerate(secs) for r in S["rows"]}
    sec_of_col = {c: i for i, S in enumerate(secs) for c in S["cols"]}
    index = {S["q"]: i for i, S in enumerate(secs)}
    dq = mpo["dq"][l + 1]
    p1 = p2 = 0
    for w1 in sorted(set(lt) & set(rt)):
        reads_l = {}
        for (tgt, src) in lt[w1]:
            reads_l.setdefault(sec_of_row[src], []).append((tgt, src))
        reads_r = {}
        for (tgt, src) in rt[w1]:
            reads_r.setdefault(sec_of_col[src], []).append((tgt, src))
        for m in sorted(set(reads_l) & set(reads_r)):
            q = secs[m]["q"]
            mp = index.get((q[0] + dq[w1][0], q[1] + dq[w1][1]))
            if mp is None:
                continue
            # the operand a product with Lt (Rt) multiplies: X_q, or T with the other side done
            ncols = secs[m]["ncols"] if order == "left" else secs[mp]["ncols"]
            nrows = secs[mp]["nrows"] if order == "left" else secs[m]["nrows"]
            for (tgt, src) in reads_l[m]:
                if sec_of_row[tgt] == mp:
                    p1 += 2 * bl[tgt[0]][2] * bl[src[0]][2] * ncols
            for (tgt, src) in reads_r[m]:
                if sec_of_col[tgt] == mp:
                    p2 += 2 * nrows * br[src[1]][2] * br[tgt[1]][2]
    return {"left": p1, "right": p2, "total": p1 + p2}
