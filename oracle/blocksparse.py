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

    def apply(self, x: dict) -> dict:
        """y = H_eff x with x, y as {(ia, s1, s2, ib): block}; loops in the canonical L, W, R order."""
        y = {k: np.zeros_like(v) for k, v in x.items()}
        for (w, w2), W12 in self.W12.items():
            Lw = self.L.get(w)
            Rw = self.R.get(w2)
            if not Lw or not Rw:
                continue
            Lby = {}
            for (iap, ia), blk in Lw.items():
                Lby.setdefault(ia, []).append((iap, blk))
            Rby = {}
            for (ibp, ib), blk in Rw.items():
                Rby.setdefault(ib, []).append((ibp, blk))
            for (ia, s1, s2, ib), xb in x.items():
                col = 4 * s1 + s2
                rows = np.nonzero(W12[:, col])[0]
                if rows.size == 0:
                    continue
                for iap, Lb in Lby.get(ia, []):
                    LX = Lb @ xb
                    for ibp, Rb in Rby.get(ib, []):
                        T = LX @ Rb.T
                        for r in rows:
                            key = (iap, r // 4, r % 4, ibp)
                            if key in y:
                                y[key] += W12[r, col] * T
        return y


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


__all__ = ["Environments", "left_environments", "right_environments", "two_site_w",
           "check_left_canonical", "check_right_canonical", "flatten", "unflatten", "dot",
           "two_site_template", "LOCAL_QN"]
