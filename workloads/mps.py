"""Seeded random matrix product states with (N, 2Sz) block structure (inputs only).

Conventions (the paper's MPS equation gives none, so they are fixed here):

* Local states of a spatial orbital, in this order: |0>, |up>, |dn>, |updn> with
  |updn> = c+_up c+_dn |0>.  Their quantum numbers (N, 2Sz) are LOCAL_QN.
* Bond j (j = 0..K) sits left of site j.  A bond sector is labelled by the quantum
  numbers of the sites left of the bond, so site j maps bond sector q to q + LOCAL_QN[s].
  Bond 0 holds (0, 0) with dimension 1, bond K holds (N, 2Sz) with dimension 1.
* Sites left of the two-site block (0..l-1) are left-canonical
  (sum_s A^s^T A^s = 1), sites right of it (l+2..K-1) are right-canonical
  (sum_s B^s B^s^T = 1).  Canonicalisation is a QR per sector with diag(R) >= 0, done
  once here so that every consumer sees the same gauge.

An MPS is a dict: n_sites, n_elec, two_sz, center (= l), bonds (list over bonds of lists of
(n, two_sz, dim)), sites (list over sites of lists of (left_sector, s, right_sector, array)).
"""
from __future__ import annotations

import numpy as np

LOCAL_QN = ((0, 0), (1, 1), (1, -1), (2, 0))


def fock_counts(n_sites: int) -> dict:
    """Number of occupation states of n_sites spatial orbitals per (N, 2Sz)."""
    counts = {(0, 0): 1}
    for _ in range(n_sites):
        nxt = {}
        for (n, sz), c in counts.items():
            for dn, dsz in LOCAL_QN:
                key = (n + dn, sz + dsz)
                nxt[key] = nxt.get(key, 0) + c
        counts = nxt
    return counts


def _apportion(weights: dict, caps: dict, total: int) -> dict:
    """Largest-remainder apportionment of `total` by `weights`, capped, repeated while caps bind."""
    alloc = {q: 0 for q in weights}
    free = sorted(q for q in weights if weights[q] > 0 and caps[q] > 0)
    remaining = total
    while free and remaining > 0:
        wsum = float(sum(weights[q] for q in free))
        raw = {q: remaining * weights[q] / wsum for q in free}
        base = {q: int(np.floor(raw[q])) for q in free}
        left = remaining - sum(base.values())
        order = sorted(free, key=lambda q: (-(raw[q] - base[q]), q))
        for q in order[:left]:
            base[q] += 1
        capped = [q for q in free if alloc[q] + base[q] >= caps[q]]
        if not capped:
            for q in free:
                alloc[q] += base[q]
            remaining = 0
            break
        for q in capped:
            remaining -= caps[q] - alloc[q]
            alloc[q] = caps[q]
        free = [q for q in free if q not in capped]
    return alloc


def allocate_bonds(n_sites: int, n_elec: int, two_sz: int, m_max: int,
                   jitter: np.ndarray | None = None) -> list:
    """Per-bond sector dimensions from Haar weights dimL(q) * dimR(Q - q).

    M_q is proportional to the weight, capped at min(dimL, dimR), summing to at most m_max;
    afterwards every sector is limited by what its neighbours can reach (so that the
    canonical QR factors have full rank).  `jitter`, if given, multiplies the weights of
    each bond (one factor per sorted sector, recycled).
    """
    Q = (n_elec, two_sz)
    bonds = []
    for j in range(n_sites + 1):
        left = fock_counts(j)
        right = fock_counts(n_sites - j)
        weights, caps = {}, {}
        for q, dl in left.items():
            qr = (Q[0] - q[0], Q[1] - q[1])
            dr = right.get(qr, 0)
            if dr > 0:
                weights[q] = float(dl) * float(dr)
                caps[q] = min(dl, dr)
        if jitter is not None and weights:
            for i, q in enumerate(sorted(weights)):
                weights[q] *= float(jitter[i % len(jitter)])
        bonds.append(_apportion(weights, caps, m_max))
    # neighbour limits, left to right then right to left, until nothing changes
    changed = True
    while changed:
        changed = False
        for j in range(n_sites):
            for q in list(bonds[j + 1]):
                reach = sum(bonds[j].get((q[0] - dn, q[1] - dsz), 0) for dn, dsz in LOCAL_QN)
                if reach < bonds[j + 1][q]:
                    bonds[j + 1][q] = reach
                    changed = True
        for j in range(n_sites, 0, -1):
            for q in list(bonds[j - 1]):
                reach = sum(bonds[j].get((q[0] + dn, q[1] + dsz), 0) for dn, dsz in LOCAL_QN)
                if reach < bonds[j - 1][q]:
                    bonds[j - 1][q] = reach
                    changed = True
    return [[(q[0], q[1], d) for q, d in sorted(b.items()) if d > 0] for b in bonds]


def _site_blocks(bond_l, bond_r):
    out = []
    index_r = {(n, sz): i for i, (n, sz, _) in enumerate(bond_r)}
    for il, (n, sz, dl) in enumerate(bond_l):
        for s, (dn, dsz) in enumerate(LOCAL_QN):
            ir = index_r.get((n + dn, sz + dsz))
            if ir is not None:
                out.append((il, s, ir))
    return out


def _left_canonical_site(sites: list, j: int) -> None:
    """Gauge step: site j becomes left-canonical (a QR per right sector, diag(R) >= 0), the
    triangular factor moves into site j+1.  The state is unchanged."""
    by_right = {}
    for blk in sites[j]:
        by_right.setdefault(blk[2], []).append(blk)
    for ir, blks in by_right.items():
        blks.sort(key=lambda b: (b[1], b[0]))
        stacked = np.concatenate([b[3] for b in blks], axis=0)
        q, r = np.linalg.qr(stacked)
        sgn = np.sign(np.diag(r))
        sgn[sgn == 0] = 1.0
        q = q * sgn
        r = sgn[:, None] * r
        off = 0
        for b in blks:
            rows = b[3].shape[0]
            b[3] = np.ascontiguousarray(q[off:off + rows])
            off += rows
        for nb in sites[j + 1]:
            if nb[0] == ir:
                nb[3] = r @ nb[3]


def _right_canonical_site(sites: list, j: int) -> None:
    """Gauge step: site j becomes right-canonical (an LQ per left sector, diag(L) >= 0), the
    triangular factor moves into site j-1.  The state is unchanged."""
    by_left = {}
    for blk in sites[j]:
        by_left.setdefault(blk[0], []).append(blk)
    for il, blks in by_left.items():
        blks.sort(key=lambda b: (b[1], b[2]))
        stacked = np.concatenate([b[3] for b in blks], axis=1)
        q, r = np.linalg.qr(stacked.T)
        sgn = np.sign(np.diag(r))
        sgn[sgn == 0] = 1.0
        q = q * sgn
        r = sgn[:, None] * r
        qt = q.T
        off = 0
        for b in blks:
            cols = b[3].shape[1]
            b[3] = np.ascontiguousarray(qt[:, off:off + cols])
            off += cols
        for pb in sites[j - 1]:
            if pb[2] == il:
                pb[3] = pb[3] @ r.T


def canonical_at(mps: dict, l: int) -> dict:
    """The same state in the gauge of the one-site problem at site l: sites 0..l-1
    left-canonical, sites l+1..K-1 right-canonical, center l."""
    sites = [[list(b) for b in blks] for blks in mps["sites"]]
    for j in range(l):
        _left_canonical_site(sites, j)
    for j in range(mps["n_sites"] - 1, l, -1):
        _right_canonical_site(sites, j)
    return dict(mps, center=l, sites=[[tuple(b) for b in blks] for blks in sites])


def one_site_gauge(mps: dict) -> dict:
    """The same state with site center+1 made right-canonical as well (its factor moves into the
    site at the center): the gauge of the one-site problem at mps['center'], whose left sites are
    left-canonical and right sites right-canonical."""
    l = mps["center"]
    sites = [[list(b) for b in blks] for blks in mps["sites"]]
    if l + 1 < mps["n_sites"]:
        _right_canonical_site(sites, l + 1)
    return dict(mps, sites=[[tuple(b) for b in blks] for blks in sites])


def random_mps(n_sites: int, n_elec: int, two_sz: int, m_max: int, seed: int,
               center: int | None = None, jitter_sigma: float = 0.0) -> dict:
    """Gaussian random MPS, left-canonical left of `center`, right-canonical right of center+1."""
    rng = np.random.Generator(np.random.PCG64(seed))
    jitter = None
    if jitter_sigma > 0:
        jitter = np.exp(jitter_sigma * rng.standard_normal(64))
    bonds = allocate_bonds(n_sites, n_elec, two_sz, m_max, jitter)
    if center is None:
        center = n_sites // 2 - 1
    sites = []
    for j in range(n_sites):
        blocks = []
        for (il, s, ir) in _site_blocks(bonds[j], bonds[j + 1]):
            a = rng.standard_normal((bonds[j][il][2], bonds[j + 1][ir][2]))
            blocks.append([il, s, ir, a])
        sites.append(blocks)
    # left-canonical sweep over sites 0..center-1
    for j in range(center):
        _left_canonical_site(sites, j)
    # right-canonical sweep over sites K-1..center+2
    for j in range(n_sites - 1, center + 1, -1):
        _right_canonical_site(sites, j)
    return {
        "n_sites": n_sites,
        "n_elec": n_elec,
        "two_sz": two_sz,
        "center": center,
        "bonds": bonds,
        "sites": [[tuple(b) for b in blks] for blks in sites],
    }


def two_site_blocks(mps: dict) -> list:
    """Allowed (left_sector, s1, s2, right_sector) blocks of the two-site tensor at the center."""
    l = mps["center"]
    bl, br = mps["bonds"][l], mps["bonds"][l + 2]
    index_r = {(n, sz): i for i, (n, sz, _) in enumerate(br)}
    out = []
    for ia, (n, sz, _) in enumerate(bl):
        for s1, (d1, z1) in enumerate(LOCAL_QN):
            for s2, (d2, z2) in enumerate(LOCAL_QN):
                ib = index_r.get((n + d1 + d2, sz + z1 + z2))
                if ib is not None:
                    out.append((ia, s1, s2, ib))
    return sorted(out)


def one_site_blocks(mps: dict) -> list:
    """Allowed (left_sector, s, right_sector) blocks of the one-site tensor at the center."""
    l = mps["center"]
    bl, br = mps["bonds"][l], mps["bonds"][l + 1]
    index_r = {(n, sz): i for i, (n, sz, _) in enumerate(br)}
    out = []
    for ia, (n, sz, _) in enumerate(bl):
        for s, (d, z) in enumerate(LOCAL_QN):
            ib = index_r.get((n + d, sz + z))
            if ib is not None:
                out.append((ia, s, ib))
    return sorted(out)


def random_one_site_vector(mps: dict, seed: int) -> dict:
    """Gaussian one-site tensor, normalised to unit 2-norm, as {(ia, s, 0, ib): array} (the key
    form of the library's one-site layout, whose second local index is the trivial 0)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    l = mps["center"]
    bl, br = mps["bonds"][l], mps["bonds"][l + 1]
    vec = {}
    for ia, s, ib in one_site_blocks(mps):
        vec[(ia, s, 0, ib)] = rng.standard_normal((bl[ia][2], br[ib][2]))
    nrm = np.sqrt(sum(float(np.sum(v * v)) for v in vec.values()))
    return {k: v / nrm for k, v in vec.items()}


def random_two_site_vector(mps: dict, seed: int) -> dict:
    """Gaussian two-site tensor, normalised to unit 2-norm, as {(ia, s1, s2, ib): array}."""
    rng = np.random.Generator(np.random.PCG64(seed))
    l = mps["center"]
    bl, br = mps["bonds"][l], mps["bonds"][l + 2]
    vec = {}
    for key in two_site_blocks(mps):
        ia, _, _, ib = key
        vec[key] = rng.standard_normal((bl[ia][2], br[ib][2]))
    nrm = np.sqrt(sum(float(np.sum(v * v)) for v in vec.values()))
    return {k: v / nrm for k, v in vec.items()}


def mps_from_amplitudes(full: np.ndarray, n_sites: int, n_elec: int, two_sz: int, tol: float = 1e-13) -> dict:
    """Exact MPS (center 0: sites 2..K-1 right-canonical) of a state given by its amplitudes over
    all 4^K site configurations (site 0 most significant, local index n_up + 2 n_dn), built by
    SVDs per (N, 2Sz) block from the right; singular values below tol * the largest are dropped.
    An input generator: it reshapes a given state, nothing of the method is computed here."""
    K = n_sites
    qn_loc = np.array(LOCAL_QN)

    def row_qn(n_rows_sites):
        # (N, 2Sz) of every configuration of sites 0..n_rows_sites-1
        q = np.zeros((1, 2), dtype=np.int64)
        for _ in range(n_rows_sites):
            q = (q[:, None, :] + qn_loc[None, :, :]).reshape(-1, 2)
        return q

    T = np.asarray(full, dtype=float).reshape(4 ** (K - 1), 4)  # rows: sites 0..K-2; cols (s, b) on bond K
    right = [(n_elec, two_sz, 1)]  # sectors of the bond right of the current site
    sites = [None] * K
    bonds = [None] * (K + 1)
    bonds[K] = right
    for j in range(K - 1, 1, -1):
        rq = row_qn(j)
        # columns (s_j, b): QN of the left part they need
        col_need = []
        off_b = np.concatenate([[0], np.cumsum([d for _, _, d in right])])
        for s in range(4):
            for ib, (n, sz, d) in enumerate(right):
                col_need.append((s, ib, n - LOCAL_QN[s][0], sz - LOCAL_QN[s][1]))
        new_sectors, blocks, Tnew_parts = [], [], []
        keys = sorted({(int(a), int(b)) for a, b in rq})
        for (qn_, qz) in keys:
            rows = np.nonzero((rq[:, 0] == qn_) & (rq[:, 1] == qz))[0]
            cols = [(s, ib) for (s, ib, n, z) in col_need if (n, z) == (qn_, qz)]
            if not cols:
                continue
            idx = np.concatenate([s * off_b[-1] + np.arange(off_b[ib], off_b[ib + 1]) for s, ib in cols])
            M = T[np.ix_(rows, idx)]
            if not np.any(M):
                continue
            U, S, Vt = np.linalg.svd(M, full_matrices=False)
            r = int(np.sum(S > tol * S[0]))
            if r == 0:
                continue
            new_sectors.append((qn_, qz, r))
            c0 = 0
            for s, ib in cols:
                d = right[ib][2]
                blocks.append([len(new_sectors) - 1, s, ib, np.ascontiguousarray(Vt[:r, c0:c0 + d])])
                c0 += d
            Tnew_parts.append((rows, U[:, :r] * S[:r]))
        bonds[j] = new_sectors
        sites[j] = [tuple(b) for b in blocks]
        width = sum(d for _, _, d in new_sectors)
        Tn = np.zeros((T.shape[0], width))
        off = 0
        for rows, blk in Tnew_parts:
            Tn[rows, off:off + blk.shape[1]] = blk
            off += blk.shape[1]
        right = new_sectors
        T = Tn.reshape(4 ** (j - 1), 4 * width)
    # sites 0 and 1 (the center block): rows s0 (bond 0 -> bond 1), columns (s1, b) on bond 2
    off_b = np.concatenate([[0], np.cumsum([d for _, _, d in right])])
    sec1, s0_blocks, s1_blocks = [], [], []
    for s0 in range(4):
        n0, z0 = LOCAL_QN[s0]
        cols = [(s1, ib) for s1 in range(4) for ib, (n, z, d) in enumerate(right)
                if (n - LOCAL_QN[s1][0], z - LOCAL_QN[s1][1]) == (n0, z0)]
        if not cols:
            continue
        idx = np.concatenate([s1 * off_b[-1] + np.arange(off_b[ib], off_b[ib + 1]) for s1, ib in cols])
        row = T[s0, idx]
        if not np.any(row):
            continue
        sec1.append((n0, z0, 1))
        s0_blocks.append([0, s0, len(sec1) - 1, np.ones((1, 1))])
        c0 = 0
        for s1, ib in cols:
            d = right[ib][2]
            s1_blocks.append([len(sec1) - 1, s1, ib, row[c0:c0 + d].reshape(1, d).copy()])
            c0 += d
    order = sorted(range(len(sec1)), key=lambda i: sec1[i][:2])
    remap = {old: new for new, old in enumerate(order)}
    bonds[1] = [sec1[i] for i in order]
    sites[0] = [(0, s, remap[r], a) for (_, s, r, a) in s0_blocks]
    sites[1] = [(remap[l], s, r, a) for (l, s, r, a) in s1_blocks]
    bonds[0] = [(0, 0, 1)]
    # bond sectors are listed in increasing (N, 2Sz) order (the keys were sorted)
    return {"n_sites": K, "n_elec": n_elec, "two_sz": two_sz, "center": 0, "bonds": bonds,
            "sites": [list(s) for s in sites]}
