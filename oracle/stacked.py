"""O2 at full size: the same environments and the same middle-bond factorisation of H_eff x
as oracle.blocksparse, with the sums over MPO channels done as matrix products.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Transition-element figure of the Implementation section: the left environment grows site by
site as
    L_{j+1}^{w'}[a', a] = sum_{w, s', s} W_j^{w,w'}[s', s] (A^{s' T} L_j^w A^s)[a', a]
(the right one mirrored).  The channels w of one bond that shift (N, 2Sz) by the same amount
have blocks on the same sector pairs, so their blocks are kept stacked, one array
(channels, rows, columns) per class and column sector; for each local pair (s', s) the
sandwich A^{s'T} L^w A^s is one batched product over the class, and the sum over w with the
MPO coefficients is a sparse matrix (w' x w) times the stack.  Nothing else is reordered: the
results are the environments of oracle.blocksparse (checked in the tests on small systems)
and the enlarged operators of its MiddleBondEnvironments.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sps

from .flops import middle_sectors
from .mpo import LOCAL_QN


def _classes(dq):
    """{shift: [channels]} and each channel's (shift, position)."""
    cls, pos = {}, {}
    for w, d in enumerate(dq):
        d = tuple(d)
        pos[w] = (d, len(cls.setdefault(d, [])))
        cls[d].append(w)
    return cls, pos


def _groups(Wj, pos_in, pos_out, cls_in, cls_out, side):
    """Sparse coefficient matrices of one site, keyed (class in, class out, s', s).

    side 'left': maps channels of the left bond onto the right bond, shape (out, in);
    side 'right': maps channels of the right bond onto the left bond."""
    acc = {}
    for (w, w2), m in Wj.items():
        d1, p1 = pos_in[w]
        d2, p2 = pos_out[w2]
        for sp in range(4):
            for s in range(4):
                c = m[sp, s]
                if c != 0.0:
                    acc.setdefault((d1, d2, sp, s), []).append((p1, p2, c))
    out = {}
    for (d1, d2, sp, s), lst in acc.items():
        r = np.array([e[1] for e in lst]) if side == "left" else np.array([e[0] for e in lst])
        c = np.array([e[0] for e in lst]) if side == "left" else np.array([e[1] for e in lst])
        v = np.array([e[2] for e in lst])
        shape = (len(cls_out[d2]), len(cls_in[d1])) if side == "left" else (len(cls_in[d1]), len(cls_out[d2]))
        out[(d1, d2, sp, s)] = sps.csr_matrix((v, (r, c)), shape=shape)
    return out


def _sector_index(bond):
    return {(n, z): i for i, (n, z, _) in enumerate(bond)}


def left_environment(mps: dict, mpo: dict, upto: int) -> dict:
    """L at bond `upto` as {shift d: {column sector a: array (channels of d, M_a', M_a)}},
    row sector a' = a shifted by d; channel order = oracle.mpo channel order within d."""
    env = {(0, 0): {0: np.ones((1, 1, 1))}}
    for j in range(upto):
        bj, bn = mps["bonds"][j], mps["bonds"][j + 1]
        ij = _sector_index(bj)
        A = {(il, s): (ir, a) for il, s, ir, a in mps["sites"][j]}
        cls_in, pos_in = _classes(mpo["dq"][j])
        cls_out, pos_out = _classes(mpo["dq"][j + 1])
        groups = _groups(mpo["W"][j], pos_in, pos_out, cls_in, cls_out, "left")
        new = {}
        for (d, d2, sp, s), Cm in groups.items():
            used = np.unique(Cm.indices)
            Cu = Cm[:, used]
            for c, E in env.get(d, {}).items():
                n, z, _ = bj[c]
                r = ij.get((n + d[0], z + d[1]))
                if r is None or (c, s) not in A or (r, sp) not in A:
                    continue
                a, As = A[(c, s)]
                ap, Asp = A[(r, sp)]
                U = np.matmul(Asp.T, np.matmul(E[used], As))  # (used, M_a', M_a)
                V = (Cu @ U.reshape(len(used), -1)).reshape(Cm.shape[0], Asp.shape[1], As.shape[1])
                tgt = new.setdefault(d2, {})
                if a in tgt:
                    tgt[a] += V
                else:
                    tgt[a] = V
        env = new
    return env


def right_environment(mps: dict, mpo: dict, fromsite: int) -> dict:
    """R at bond `fromsite` as {shift d: {column sector b: array (channels of d, M_b', M_b)}},
    row sector b' = b shifted by d."""
    K = mps["n_sites"]
    env = {(0, 0): {0: np.ones((1, 1, 1))}}
    for j in range(K - 1, fromsite - 1, -1):
        bn = mps["bonds"][j + 1]
        inn = _sector_index(bn)
        B = {(ir, s): (il, a) for il, s, ir, a in mps["sites"][j]}
        cls_l, pos_l = _classes(mpo["dq"][j])
        cls_r, pos_r = _classes(mpo["dq"][j + 1])
        groups = _groups(mpo["W"][j], pos_l, pos_r, cls_l, cls_r, "right")  # (d_left, d_right, s', s): (left, right)
        new = {}
        for (d, d2, sp, s), Cm in groups.items():
            used = np.unique(Cm.indices)
            Cu = Cm[:, used]
            for c, E in env.get(d2, {}).items():
                n, z, _ = bn[c]
                cp = inn.get((n + d2[0], z + d2[1]))
                if cp is None or (c, s) not in B or (cp, sp) not in B:
                    continue
                b, Bs = B[(c, s)]
                bp, Bsp = B[(cp, sp)]
                U = np.matmul(Bsp, np.matmul(E[used], Bs.T))  # (used, M_b', M_b)
                V = (Cu @ U.reshape(len(used), -1)).reshape(Cm.shape[0], Bsp.shape[0], Bs.shape[0])
                tgt = new.setdefault(d, {})
                if b in tgt:
                    tgt[b] += V
                else:
                    tgt[b] = V
        env = new
    return env


def as_blocks(env: dict, dq: list, bond: list) -> dict:
    """Stacked environment -> oracle.blocksparse's {w: {(row sector, column sector): block}}.
    Every channel of a class gets a block on every sector pair of the class; where no term of
    the channel reaches that pair the block is zero."""
    cls, _ = _classes(dq)
    idx = _sector_index(bond)
    out = {}
    for d, per in env.items():
        for c, E in per.items():
            n, z, _ = bond[c]
            r = idx[(n + d[0], z + d[1])]
            for k, w in enumerate(cls[d]):
                out.setdefault(w, {})[(r, c)] = E[k]
    return out


class FullSizeEnvironments:
    """H_eff x = sum_{w1} Lt^{w1} X Rt^{w1 T} (the factorisation of
    oracle.blocksparse.MiddleBondEnvironments) on stacked environments."""

    def __init__(self, spec: dict, mps: dict, mpo: dict):
        l = self.l = mps["center"]
        self.bl, self.br = mps["bonds"][l], mps["bonds"][l + 2]
        self.dq = mpo["dq"][l + 1]
        self.secs = middle_sectors(mps)
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
        L = left_environment(mps, mpo, l)
        R = right_environment(mps, mpo, l + 2)
        self.lt = self._enlarge(L, mpo["W"][l], mpo["dq"][l], mpo["dq"][l + 1], self.bl, "left")
        del L
        self.rt = self._enlarge(R, mpo["W"][l + 1], mpo["dq"][l + 1], mpo["dq"][l + 2], self.br, "right")

    def _enlarge(self, E, Wsite, dq_a, dq_b, bond, side):
        """lt[w1][((a',s1'),(a,s1))] = sum_w W_l^{w,w1}[s1',s1] L^w[a',a]   (side 'left'), or
        rt[w1][((s2',b'),(s2,b))] = sum_w2 W_{l+1}^{w1,w2}[s2',s2] R^w2[b',b]  (side 'right')."""
        cls_a, pos_a = _classes(dq_a)
        cls_b, pos_b = _classes(dq_b)
        idx = _sector_index(bond)
        groups = _groups(Wsite, pos_a, pos_b, cls_a, cls_b, side)
        mid_cls = cls_b if side == "left" else cls_a
        out = {}
        for (da, db, sp, s), Cm in groups.items():
            d_env, d_mid = (da, db) if side == "left" else (db, da)
            rows = np.unique(Cm.tocoo().row)
            Cr = Cm[rows, :]
            for c, Ec in E.get(d_env, {}).items():
                n, z, _ = bond[c]
                r = idx.get((n + d_env[0], z + d_env[1]))
                if side == "left":
                    tgt, src = (r, sp), (c, s)
                    ok = tgt in self.row_at and src in self.row_at
                else:
                    tgt, src = (sp, r), (s, c)
                    ok = tgt in self.col_at and src in self.col_at
                if not ok:
                    continue
                V = (Cr @ Ec.reshape(Ec.shape[0], -1)).reshape(len(rows), Ec.shape[1], Ec.shape[2])
                for k, rw in enumerate(rows):
                    w1 = mid_cls[d_mid][rw]
                    out.setdefault(w1, {})[(tgt, src)] = V[k]
        return out

    def to_sectors(self, x: dict) -> list:
        out = [np.zeros((S["nrows"], S["ncols"])) for S in self.secs]
        for (a, s1, s2, b), blk in x.items():
            i, r0 = self.row_at[(a, s1)]
            _, c0 = self.col_at[(s2, b)]
            out[i][r0:r0 + blk.shape[0], c0:c0 + blk.shape[1]] = blk
        return out

    def from_sectors(self, ys: list, template: dict) -> dict:
        out = {}
        for (a, s1, s2, b), blk in template.items():
            i, r0 = self.row_at[(a, s1)]
            _, c0 = self.col_at[(s2, b)]
            out[(a, s1, s2, b)] = ys[i][r0:r0 + blk.shape[0], c0:c0 + blk.shape[1]].copy()
        return out

    def apply_sectors(self, X: list, channels=None, counter: dict | None = None) -> list:
        """Y = H_eff X on per-sector matrices (all middle channels, or the given subset);
        `counter`, if given, receives the multiply-add work done (2 per multiply-add) as
        counter['flops']."""
        cnt = counter if counter is not None else {}
        cnt.setdefault("flops", 0)
        Y = [np.zeros_like(m) for m in X]
        index = {S["q"]: i for i, S in enumerate(self.secs)}
        chans = sorted(set(self.lt) & set(self.rt)) if channels is None else channels
        for w1 in chans:
            lt, rt = self.lt.get(w1, {}), self.rt.get(w1, {})
            src_l = {self.row_at[src][0] for (_, src) in lt}
            src_r = {self.col_at[src][0] for (_, src) in rt}
            for m in sorted(src_l & src_r):
                q = self.secs[m]["q"]
                mp = index.get((q[0] + self.dq[w1][0], q[1] + self.dq[w1][1]))
                if mp is None:
                    continue
                T = np.zeros((self.secs[mp]["nrows"], self.secs[m]["ncols"]))
                for (tgt, src), blk in lt.items():
                    i, r0 = self.row_at[src]
                    if i != m:
                        continue
                    _, t0 = self.row_at[tgt]
                    T[t0:t0 + blk.shape[0], :] += blk @ X[m][r0:r0 + blk.shape[1], :]
                    cnt["flops"] += 2 * blk.shape[0] * blk.shape[1] * T.shape[1]
                for (tgt, src), blk in rt.items():
                    j, c0 = self.col_at[src]
                    if j != m:
                        continue
                    _, d0 = self.col_at[tgt]
                    Y[mp][:, d0:d0 + blk.shape[0]] += T[:, c0:c0 + blk.shape[1]] @ blk.T
                    cnt["flops"] += 2 * T.shape[0] * blk.shape[1] * blk.shape[0]
        return Y

    def apply(self, x: dict) -> dict:
        return self.from_sectors(self.apply_sectors(self.to_sectors(x)), x)
