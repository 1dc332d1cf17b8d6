"""The oracle's matrix product operator: a plain prefix automaton (MPO equation).

The MPO equation writes an operator as a product of site tensors W^{n n'} contracted over
virtual (channel) indices.  The oracle builds one in the most literal way:

* every operator string of H (oracle.fock.operator_strings) is sorted by site with the
  fermionic sign of the permutation, and its factors are turned into site-local 4x4
  matrices with Jordan-Wigner strings: a factor at site t is
      (product of the string's operators that sit at t) @ F^(number of operators right of t)
  with F = diag(1,-1,-1,1) the local parity;
* the channel of a string at bond j (left of site j) is its prefix (the operators on sites
  < j), or "H" once the string is complete; the coefficient is applied on completion.

No compression, no complementary operators: the bond dimension is the number of distinct
incomplete prefixes, which is only affordable for small systems with two-body terms and
for any size with one-body + on-site terms.  Exactness is by construction; it is pinned
against the Fock-space Hamiltonian in the tests.
"""
from __future__ import annotations

import numpy as np

from . import fock

# local basis |0>, |up>, |dn>, |updn>, |updn> = c+_up c+_dn |0>
_CDAG_UP = np.zeros((4, 4))
_CDAG_UP[1, 0] = 1.0
_CDAG_UP[3, 2] = 1.0
_CDAG_DN = np.zeros((4, 4))
_CDAG_DN[2, 0] = 1.0
_CDAG_DN[3, 1] = -1.0  # c+_dn |up> = c+_dn c+_up |0> = -|updn>
F = np.diag([1.0, -1.0, -1.0, 1.0])
ID = np.eye(4)
LOCAL_QN = ((0, 0), (1, 1), (1, -1), (2, 0))


def local_op(spin: int, dagger: bool) -> np.ndarray:
    m = _CDAG_UP if spin == 0 else _CDAG_DN
    return m if dagger else m.T


def _site_strings(spec: dict):
    """(coefficient with reordering sign, [(site, spin, dagger), ...] sorted by site)."""
    for coef, ops in fock.operator_strings(spec):
        items = [(p // 2, p % 2, dag) for p, dag in ops]
        order = sorted(range(len(items)), key=lambda i: items[i][0])  # stable
        # parity of the permutation `order`
        perm = list(order)
        sign = 1.0
        seen = [False] * len(perm)
        for i in range(len(perm)):
            if not seen[i]:
                j, cyc = i, 0
                while not seen[j]:
                    seen[j] = True
                    j = perm[j]
                    cyc += 1
                if cyc % 2 == 0:
                    sign = -sign
        yield coef * sign, [items[i] for i in order]


def _dq(prefix) -> tuple:
    dn = dz = 0
    for _, spin, dag in prefix:
        s = 1 if dag else -1
        dn += s
        dz += s * (1 if spin == 0 else -1)
    return (dn, dz)


def build_mpo(spec: dict) -> dict:
    """Return {'channels': [list of labels per bond 0..K], 'dq': [...], 'W': [dict per site]}.

    W[j][(w_in, w_out)] is the 4x4 matrix <s'|.|s> for channel w_in at bond j and w_out at
    bond j+1.  Bond 0 holds the single channel () and bond K the single channel 'H'.
    """
    K = spec["n_orb"]
    entries = [dict() for _ in range(K)]  # label pairs -> matrix
    fixed = [dict() for _ in range(K)]

    def put(j, a, b, mat, add):
        if add:
            entries[j][(a, b)] = entries[j].get((a, b), 0.0) + mat
        else:
            old = fixed[j].get((a, b))
            if old is not None:
                assert np.array_equal(old, mat), "inconsistent prefix transition"
            fixed[j][(a, b)] = mat

    for coef, ops in _site_strings(spec):
        nops = len(ops)
        last = ops[-1][0]
        for j in range(last + 1):
            before = tuple(o for o in ops if o[0] < j)
            here = [o for o in ops if o[0] == j]
            after_count = sum(1 for o in ops if o[0] > j)
            mat = ID.copy()
            for _, spin, dag in here:
                mat = mat @ local_op(spin, dag)
            if after_count % 2 == 1:
                mat = mat @ F
            if j == last:
                put(j, before, "H", coef * mat, True)
            else:
                put(j, before, before + tuple(here), mat, False)
    if spec.get("e_const", 0.0) != 0.0:
        put(0, (), "H", spec["e_const"] * ID, True)
    # channel sets per bond
    chans = [set() for _ in range(K + 1)]
    chans[0].add(())
    chans[K].add("H")
    for j in range(K):
        for (a, b) in list(entries[j]) + list(fixed[j]):
            chans[j].add(a)
            chans[j + 1].add(b)
    # H passes through with the identity
    for j in range(1, K):
        if "H" in chans[j]:
            put(j, "H", "H", ID, False)
            chans[j + 1].add("H")

    def key(lab):
        return (1, ()) if lab == "H" else (0, (len(lab), lab))

    labels = [sorted(c, key=key) for c in chans]
    index = [{lab: i for i, lab in enumerate(ls)} for ls in labels]
    W = []
    for j in range(K):
        d = {}
        for (a, b), m in list(fixed[j].items()) + list(entries[j].items()):
            k = (index[j][a], index[j + 1][b])
            d[k] = d.get(k, 0.0) + m
        W.append(d)
    dq = [[(0, 0) if lab == "H" else _dq(lab) for lab in ls] for ls in labels]
    return {"channels": labels, "dq": dq, "W": W, "n_sites": K}


def dense_operator(mpo: dict) -> np.ndarray:
    """Contract the MPO to a dense 4^K x 4^K matrix (site 0 most significant).  Tiny K only."""
    K = mpo["n_sites"]
    # partial[w] = operator on sites 0..j-1 for channel w at bond j
    partial = {0: np.ones((1, 1))}
    for j in range(K):
        nxt = {}
        for (a, b), m in mpo["W"][j].items():
            if a in partial:
                nxt[b] = nxt.get(b, 0.0) + np.kron(partial[a], m)
        partial = nxt
    return partial[0]
