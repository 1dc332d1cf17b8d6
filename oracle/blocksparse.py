"""O2: block-sparse environments and the two-site H_eff x, plain FP64 numpy.

Transition-element figure and the local-derivative figure of the Implementation section:
<Psi|H|Phi> is contracted site by site through MPS and MPO tensors; removing the two-site
tensor leaves a left environment L (sites < l), the MPO tensors of sites l and l+1, and a
right environment R (sites > l+1).  Applied to a two-site tensor x:

  y[a',s1',s2',b'] = sum_{w,w2,s1,s2,a,b} W12^{w,w2}[s1's2', s1s2] L^w[a',a] x[a,s1,s2,b] R^{w2}[b',b]
  W12^{w,w2} = sum_{w1} W_l^{w,w1} (x) W_{l+1}^{w1,w2}

Environments are dicts: env[w] = {(sector', sector): block}; blocks follow the (N, 2Sz)
selection rule sector' = sector + dq(w) (sectors are bond labels, see workloads.mps).
"""
from __future__ import annotations

import numpy as np

from .mpo import LOCAL_QN


def _site_index(blocks):
    """{(left_sector, s): (right_sector, array)}."""
    return {(il, s): (ir, a) for il, s, ir, a in blocks}


def left_environments(mps: dict, mpo: dict, upto: int) -> dict:
    """L at bond `upto` (operators on sites 0..upto-1): L[w][(ia', ia)] = <a'|O^w_L|a>."""
    env = {0: {(0, 0): np.ones((1, 1))}}
    for j in range(upto):
        A = _site_index(mps["sites"][j])
        new = {}
        for (w, w2), Wm in mpo["W"][j].items():
            if w not in env:
                continue
            nz = [(sp, s) for sp in range(4) for s in range(4) if Wm[sp, s] != 0.0]
            for (ibp, ib), Lb in env[w].items():
                for sp, s in nz:
                    ka = A.get((ib, s))
                    kp = A.get((ibp, sp))
                    if ka is None or kp is None:
                        continue
                    ia, Aa = ka
                    iap, Ap = kp
                    blk = Wm[sp, s] * (Ap.T @ Lb @ Aa)
                    tgt = new.setdefault(w2, {})
                    if (iap, ia) in tgt:
                        tgt[(iap, ia)] = tgt[(iap, ia)] + blk
                    else:
                        tgt[(iap, ia)] = blk
        env = new
    return env


def right_environments(mps: dict, mpo: dict, fromsite: int) -> dict:
    """R at bond `fromsite` (operators on sites fromsite..K-1): R[w][(ib', ib)] = <b'|O^w_R|b>."""
    K = mps["n_sites"]
    nb = len(mpo["channels"][K])
    assert nb == 1
    env = {0: {(0, 0): np.ones((1, 1))}}
    for j in range(K - 1, fromsite - 1, -1):
        B = {}
        for il, s, ir, a in mps["sites"][j]:
            B[(ir, s)] = (il, a)
        new = {}
        for (w, w2), Wm in mpo["W"][j].items():
            if w2 not in env:
                continue
            nz = [(sp, s) for sp in range(4) for s in range(4) if Wm[sp, s] != 0.0]
            for (icp, ic), Rb in env[w2].items():
                for sp, s in nz:
                    kb = B.get((ic, s))
                    kp = B.get((icp, sp))
                    if kb is None or kp is None:
                        continue
                    ib, Bb = kb
                    ibp, Bp = kp
                    blk = Wm[sp, s] * (Bp @ Rb @ Bb.T)
                    tgt = new.setdefault(w, {})
                    if (ibp, ib) in tgt:
                        tgt[(ibp, ib)] = tgt[(ibp, ib)] + blk
                    else:
                        tgt[(ibp, ib)] = blk
        env = new
    return env


def two_site_w(mpo: dict, l: int) -> dict:
    """W12[(w, w2)] as a 16x16 matrix over (s1 s2) = 4*s1 + s2, summed over the middle bond."""
    out = {}
    right = {}
    for (w1, w2), m2 in mpo["W"][l + 1].items():
        right.setdefault(w1, []).append((w2, m2))
    for (w, w1), m1 in mpo["W"][l].items():
        for w2, m2 in right.get(w1, []):
            k = np.kron(m1, m2)
            out[(w, w2)] = out.get((w, w2), 0.0) + k
    return out


class Environments:
    """Everything the oracle needs to apply H_eff at the two-site block of `mps`."""

    def __init__(self, spec: dict, mps: dict, mpo: dict):
        self.mps = mps
        self.l = mps["center"]
        self.L = left_environments(mps, mpo, self.l)
        self.R = right_environments(mps, mpo, self.l + 2)
        self.W12 = two_site_w(mpo, self.l)

    def apply(self, x: dict, counter: dict | None = None) -> dict:
        """y = H_eff x with x, y as {(ia, s1, s2, ib): block}, in the canonical order:
        K1 T_w = L^w X, K2 Z_w2 = sum W12^{w,w2} T_w, K3 y += Z_w2 R^{w2 T}.

        Only work that reaches an allowed y block is done: the Z blocks are the ones some R
        block carries into y, and a T block is formed the first time a nonzero W12 entry asks
        for it.  `counter`, if given, receives the multiply-add work as counter['k1'],
        counter['k2'], counter['k3'] (2 per multiply-add)."""
        cnt = counter if counter is not None else {}
        for k in ("k1", "k2", "k3"):
            cnt.setdefault(k, 0)
        y = {k: np.zeros_like(v) for k, v in x.items()}
        # L^w by row sector: for a fixed channel the source sector follows from the row
        lrow = {w: {iap: (ia, blk) for (iap, ia), blk in Lw.items()} for w, Lw in self.L.items()}
        # y blocks by right sector, and the Z blocks each R^{w2} needs
        y_by_right = {}
        for (ia, s1, s2, ib) in y:
            y_by_right.setdefault(ib, []).append((ia, s1, s2))
        z_need = {}
        for w2, Rw in self.R.items():
            need = set()
            for (ibp, ib) in Rw:
                for (iap, s1p, s2p) in y_by_right.get(ibp, []):
                    need.add((iap, s1p, s2p, ib))
            z_need[w2] = sorted(need)
        T = {}

        def get_t(w, iap, s1, s2, ib):
            key = (w, iap, s1, s2, ib)
            if key not in T:
                hit = lrow.get(w, {}).get(iap)
                xb = None if hit is None else x.get((hit[0], s1, s2, ib))
                if xb is None:
                    T[key] = None
                else:
                    T[key] = hit[1] @ xb
                    cnt["k1"] += 2 * hit[1].shape[0] * hit[1].shape[1] * xb.shape[1]
            return T[key]

        Z = {}
        for (w, w2), W12 in self.W12.items():
            if w not in self.L or w2 not in self.R:
                continue
            for (iap, s1p, s2p, ib) in z_need[w2]:
                row = 4 * s1p + s2p
                for col in np.nonzero(W12[row, :])[0]:
                    t = get_t(w, iap, col // 4, col % 4, ib)
                    if t is None:
                        continue
                    zk = (w2, iap, s1p, s2p, ib)
                    if zk in Z:
                        Z[zk] = Z[zk] + W12[row, col] * t
                    else:
                        Z[zk] = W12[row, col] * t
                    cnt["k2"] += 2 * t.size
        for (w2, iap, s1p, s2p, ib), z in Z.items():
            for (ibp, ib2), Rb in self.R[w2].items():
                key = (iap, s1p, s2p, ibp)
                if ib2 == ib and key in y:
                    y[key] += z @ Rb.T
                    cnt["k3"] += 2 * z.shape[0] * z.shape[1] * Rb.shape[0]
        return y


class MiddleBondEnvironments:
    """H_eff x factorised over the middle MPO bond (transition-element figure, cut between the
    two sites): H_eff = sum_{w1} Lt^{w1} (x) Rt^{w1} with
        Lt^{w1}[(a',s1'),(a,s1)] = sum_w  W_l^{w,w1}[s1',s1] L^w[a',a]
        Rt^{w1}[(s2',b'),(s2,b)] = sum_w2 W_{l+1}^{w1,w2}[s2',s2] R^{w2}[b',b].
    The two-site vector is one matrix X_q per middle-bond sector q (rows (a, s1), columns
    (s2, b)), so that y is Y_{q'} = sum_{w1} Lt^{w1} X_q Rt^{w1 T} with q' = q + dq(w1)."""

    def __init__(self, spec: dict, mps: dict, mpo: dict, one_site: bool = False):
        """one_site: the problem of the site tensor at the center (columns b of the next bond,
        written (0, b); Rt^{w1} = R^{w1}, the right environment of the sites right of it)."""
        from .flops import middle_sectors
        self.mps = mps
        l = self.l = mps["center"]
        self.bl, self.br = mps["bonds"][l], mps["bonds"][l + (1 if one_site else 2)]
        self.dq = mpo["dq"][l + 1]
        L = left_environments(mps, mpo, l)
        R = right_environments(mps, mpo, l + (1 if one_site else 2))
        self.secs = middle_sectors(mps, one_site)
        self.row_at, self.col_at = {}, {}
        for i, S in enumerate(self.secs):
            off = 0
            for (a, s1) in S["rows"]:
                self.row_at[(a, s1)] = (i, off)
                off += self.bl[a][2]
            off = 0
            for (s2, b) in S["cols"]:
                self.col_at[(s2, b)] = (i, off)
                off += self.br[b][2]
        self.lt, self.rt = {}, {}
        for (w, w1), m in mpo["W"][l].items():
            for (ap, a), blk in L.get(w, {}).items():
                for sp in range(4):
                    for s in range(4):
                        if m[sp, s] != 0.0 and (ap, sp) in self.row_at and (a, s) in self.row_at:
                            key = ((ap, sp), (a, s))
                            d = self.lt.setdefault(w1, {})
                            d[key] = d.get(key, 0.0) + m[sp, s] * blk
        if one_site:
            for w1, blocks in R.items():
                for (bp, b), blk in blocks.items():
                    if (0, bp) in self.col_at and (0, b) in self.col_at:
                        self.rt.setdefault(w1, {})[((0, bp), (0, b))] = blk
            return
        for (w1, w2), m in mpo["W"][l + 1].items():
            for (bp, b), blk in R.get(w2, {}).items():
                for sp in range(4):
                    for s in range(4):
                        if m[sp, s] != 0.0 and (sp, bp) in self.col_at and (s, b) in self.col_at:
                            key = ((sp, bp), (s, b))
                            d = self.rt.setdefault(w1, {})
                            d[key] = d.get(key, 0.0) + m[sp, s] * blk

    def to_sectors(self, x: dict) -> list:
        out = [np.zeros((S["nrows"], S["ncols"])) for S in self.secs]
        for (a, s1, s2, b), blk in x.items():
            i, r0 = self.row_at[(a, s1)]
            j, c0 = self.col_at[(s2, b)]
            assert i == j
            out[i][r0:r0 + blk.shape[0], c0:c0 + blk.shape[1]] = blk
        return out

    def from_sectors(self, ys: list, template: dict) -> dict:
        out = {}
        for (a, s1, s2, b), blk in template.items():
            i, r0 = self.row_at[(a, s1)]
            _, c0 = self.col_at[(s2, b)]
            out[(a, s1, s2, b)] = ys[i][r0:r0 + blk.shape[0], c0:c0 + blk.shape[1]].copy()
        return out

    def apply(self, x: dict, counter: dict | None = None, order: str = "left") -> dict:
        """y = H_eff x, per (w1, q) pair where Lt^{w1} and Rt^{w1} both read sector q and
        q' = q + dq(w1) is a sector.  order "left": T = Lt^{w1} X_q, then Y_q' += T Rt^{w1 T};
        order "right": T = X_q Rt^{w1 T}, then Y_q' += Lt^{w1} T.  `counter` receives the
        multiply-add work of the products with the enlarged left operator as counter['left']
        and with the enlarged right operator as counter['right']."""
        if order not in ("left", "right"):
            raise ValueError(order)
        cnt = counter if counter is not None else {}
        cnt.setdefault("left", 0)
        cnt.setdefault("right", 0)
        X = self.to_sectors(x)
        Y = [np.zeros_like(m) for m in X]
        index = {S["q"]: i for i, S in enumerate(self.secs)}
        for w1 in sorted(set(self.lt) & set(self.rt)):
            src_l = {self.row_at[src][0] for (_, src) in self.lt[w1]}
            src_r = {self.col_at[src][0] for (_, src) in self.rt[w1]}
            for m in sorted(src_l & src_r):
                q = self.secs[m]["q"]
                mp = index.get((q[0] + self.dq[w1][0], q[1] + self.dq[w1][1]))
                if mp is None:
                    continue
                lt = [(self.row_at[tgt][1], self.row_at[src][1], blk)
                      for (tgt, src), blk in self.lt[w1].items() if self.row_at[src][0] == m]
                rt = [(self.col_at[tgt][1], self.col_at[src][1], blk)
                      for (tgt, src), blk in self.rt[w1].items() if self.col_at[src][0] == m]
                if order == "left":
                    T = np.zeros((self.secs[mp]["nrows"], self.secs[m]["ncols"]))
                    for t0, r0, blk in lt:
                        T[t0:t0 + blk.shape[0], :] += blk @ X[m][r0:r0 + blk.shape[1], :]
                        cnt["left"] += 2 * blk.shape[0] * blk.shape[1] * X[m].shape[1]
                    for d0, c0, blk in rt:
                        Y[mp][:, d0:d0 + blk.shape[0]] += T[:, c0:c0 + blk.shape[1]] @ blk.T
                        cnt["right"] += 2 * T.shape[0] * blk.shape[1] * blk.shape[0]
                else:
                    T = np.zeros((self.secs[m]["nrows"], self.secs[mp]["ncols"]))
                    for d0, c0, blk in rt:
                        T[:, d0:d0 + blk.shape[0]] += X[m][:, c0:c0 + blk.shape[1]] @ blk.T
                        cnt["right"] += 2 * X[m].shape[0] * blk.shape[1] * blk.shape[0]
                    for t0, r0, blk in lt:
                        Y[mp][t0:t0 + blk.shape[0], :] += blk @ T[r0:r0 + blk.shape[1], :]
                        cnt["left"] += 2 * blk.shape[0] * blk.shape[1] * T.shape[1]
        return self.from_sectors(Y, x)


def check_left_canonical(mps: dict, tol: float = 1e-12) -> float:
    """max |sum_s A^s^T A^s - 1| over sites left of the two-site block."""
    worst = 0.0
    for j in range(mps["center"]):
        acc = {}
        for il, s, ir, a in mps["sites"][j]:
            acc[ir] = acc.get(ir, 0.0) + a.T @ a
        for ir, m in acc.items():
            worst = max(worst, float(np.abs(m - np.eye(m.shape[0])).max()))
    return worst


def check_right_canonical(mps: dict) -> float:
    worst = 0.0
    for j in range(mps["center"] + 2, mps["n_sites"]):
        acc = {}
        for il, s, ir, a in mps["sites"][j]:
            acc[il] = acc.get(il, 0.0) + a @ a.T
        for il, m in acc.items():
            worst = max(worst, float(np.abs(m - np.eye(m.shape[0])).max()))
    return worst


def flatten(vec: dict, blocks: list) -> np.ndarray:
    """Concatenate blocks in `blocks` order, row-major inside each block (the O1 column order)."""
    return np.concatenate([vec[k].reshape(-1) for k in blocks])


def unflatten(arr: np.ndarray, template: dict, blocks: list) -> dict:
    out, off = {}, 0
    for k in blocks:
        shp = template[k].shape
        n = shp[0] * shp[1]
        out[k] = arr[off:off + n].reshape(shp).copy()
        off += n
    return out


def dot(a: dict, b: dict) -> float:
    return float(sum(np.sum(a[k] * b[k]) for k in a))


def two_site_template(mps: dict, blocks: list) -> dict:
    l = mps["center"]
    bl, br = mps["bonds"][l], mps["bonds"][l + 2]
    return {k: np.zeros((bl[k[0]][2], br[k[3]][2])) for k in blocks}


def one_site_embed(mps: dict, x1: dict, two_site_keys: list) -> dict:
    """E x1: the two-site tensor of the block (c, c+1), c = mps['center'], that a one-site tensor
    x1 at c represents with the right-canonical site c+1 of mps fixed,
        x2[a, s1, s2, b'] = sum_b x1[a, s1, b] B^{s2}[b, b'],
    so that the one-site isometry is the two-site one times E (P1 = P2 E).  x1 is keyed
    (a, s1, 0, b)."""
    c = mps["center"]
    bl, br = mps["bonds"][c], mps["bonds"][c + 2]
    x2 = {k: np.zeros((bl[k[0]][2], br[k[3]][2])) for k in two_site_keys}
    for (a, s1, _, b), blk in x1.items():
        for (il, s2, ir, B) in mps["sites"][c + 1]:
            if il == b and (a, s1, s2, ir) in x2:
                x2[(a, s1, s2, ir)] += blk @ B
    return x2


def one_site_contract(mps: dict, y2: dict, one_site_keys: list) -> dict:
    """E^T y2: y1[a, s1, b] = sum_{s2, b'} y2[a, s1, s2, b'] B^{s2}[b, b']^T."""
    c = mps["center"]
    bl, bm = mps["bonds"][c], mps["bonds"][c + 1]
    y1 = {k: np.zeros((bl[k[0]][2], bm[k[3]][2])) for k in one_site_keys}
    for (il, s2, ir, B) in mps["sites"][c + 1]:
        for (a, s1, _, b) in one_site_keys:
            if b == il and (a, s1, s2, ir) in y2:
                y1[(a, s1, 0, b)] += y2[(a, s1, s2, ir)] @ B.T
    return y1


def one_site_apply(spec: dict, mps: dict, mpo: dict, x1: dict) -> dict:
    """y = H1 x1 for the site tensor at mps['center'] (sites left of it left-canonical, right of
    it right-canonical): H1 = P1^T H P1 = E^T (P2^T H P2) E, the two-site H_eff of (c, c+1) of
    `Environments` between the embedding and its transpose.  Needs c + 1 < K."""
    from workloads import mps as M  # block enumeration of the generator (inputs only)
    keys2 = M.two_site_blocks(mps)
    y2 = Environments(spec, mps, mpo).apply(one_site_embed(mps, x1, keys2))
    return one_site_contract(mps, y2, sorted(x1))


__all__ = ["Environments", "MiddleBondEnvironments", "left_environments", "right_environments", "two_site_w",
           "check_left_canonical", "check_right_canonical", "flatten", "unflatten", "dot",
           "two_site_template", "one_site_embed", "one_site_contract", "one_site_apply", "LOCAL_QN"]
