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

import bisect

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
    if fock.constant(spec) != 0.0:
        put(0, (), "H", fock.constant(spec) * ID, True)
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


def build_mpo_twosided(spec: dict, switch: int | None = None) -> dict:
    """An exact MPO whose bond dimension stays O(k^2) for two-body terms (MPO equation; the
    Implementation section bounds it by k^2 with spin adaptation, this one uses spin orbitals).

    Each operator string is sorted by site with the sign of the permutation, as in build_mpo.
    At bond j it splits into the operators left of j (nL of them) and right of j (nR).  The
    channel that carries it is labelled by whichever side is shorter:
        nL = 0: 'I'        nR = 0: 'H'
        nL < nR: ('L', left operators)    the coefficient has not been applied yet
        nL > nR: ('R', right operators)   the coefficient has been applied
        nL = nR = 1: ('R', right operator)
        nL = nR = 2: ('L', ...) on bonds j < switch, ('R', ...) on bonds j >= switch
    so no label holds more than two operators.  The coefficient enters on the one transition
    from an 'I' / 'L' channel into an 'R' / 'H' channel; every other transition is fixed by the
    labels.  On a site where a string has no operator its channel passes through with the
    local parity F^(number of its operators on the far side), the Jordan-Wigner string.
    `switch` defaults to k // 2.  Same output format as build_mpo.
    """
    K = spec["n_orb"]
    sw = K // 2 if switch is None else switch

    def label(ops, j):
        nl = bisect.bisect_left(ops, (j,))  # operators on sites < j (ops are sorted by site)
        nr = len(ops) - nl
        if nl == 0:
            return "I"
        if nr == 0:
            return "H"
        if nl < nr or (nl == nr == 2 and j < sw):
            return ("L",) + tuple(ops[:nl])
        return ("R",) + tuple(ops[nl:])

    def applies_coefficient(a, b):
        return (a == "I" or a[0] == "L") and (b == "H" or b[0] == "R")

    coef_entries = [dict() for _ in range(K)]
    fixed = [dict() for _ in range(K)]
    first, last = {}, {}

    def seen(lab, b0, b1):
        first[lab] = min(first.get(lab, b0), b0)
        last[lab] = max(last.get(lab, b1), b1)

    # identical site-sorted strings (e.g. the (ij|kl) and (kl|ij) images) are merged first
    merged = {}
    for coef, ops in _site_strings(spec):
        key = tuple(ops)
        merged[key] = merged.get(key, 0.0) + coef
    for ops, coef in merged.items():
        if coef == 0.0:
            continue
        sites = sorted({o[0] for o in ops})
        local = {}
        for t in sites:
            m = ID.copy()
            for _, spin, dag in (o for o in ops if o[0] == t):
                m = m @ local_op(spin, dag)
            local[t] = m
        if any(not np.any(m) for m in local.values()):
            continue  # e.g. a+_p a+_p: the zero operator
        events = sorted(set(sites) | ({sw - 1} if 0 <= sw - 1 < K else set()))
        # bond ranges of the string's labels: constant between consecutive events
        b0 = 0
        for e in events:
            seen(label(ops, b0), b0, e)
            b0 = e + 1
        seen(label(ops, b0), b0, K)
        for j in events:
            a, b = label(ops, j), label(ops, j + 1)
            if j not in local and a == b:
                continue  # plain pass-through, added per channel below
            m = local.get(j, ID)
            if (len(ops) - bisect.bisect_left(ops, (j + 1,))) % 2 == 1:  # operators right of site j
                m = m @ F
            if applies_coefficient(a, b):
                coef_entries[j][(a, b)] = coef_entries[j].get((a, b), 0.0) + coef * m
            else:
                old = fixed[j].get((a, b))
                assert old is None or np.array_equal(old, m), "inconsistent label transition"
                fixed[j][(a, b)] = m
    if fock.constant(spec) != 0.0:
        coef_entries[0][("I", "H")] = coef_entries[0].get(("I", "H"), 0.0) + fock.constant(spec) * ID
        seen("I", 0, 0)
        seen("H", 1, K)
    # pass-through of every channel inside its range of bonds
    for lab in first:
        par = F if (lab not in ("I", "H") and (len(lab) - 1) % 2 == 1) else ID
        for j in range(first[lab], last[lab]):
            old = fixed[j].get((lab, lab))
            assert old is None or np.array_equal(old, par), "inconsistent pass-through"
            fixed[j][(lab, lab)] = par

    def order(lab):
        if lab == "I":
            return (0, ())
        if lab == "H":
            return (1, ())
        return (2 if lab[0] == "L" else 3, (len(lab), lab[1:]))

    chans = [sorted((lab for lab in first if first[lab] <= b <= last[lab]), key=order) for b in range(K + 1)]
    assert chans[0] == ["I"] and chans[K] == ["H"], "boundary bonds must hold one channel"
    index = [{lab: i for i, lab in enumerate(c)} for c in chans]

    def shift(lab):
        if lab in ("I", "H"):
            return (0, 0)
        dn, dz = _dq(lab[1:])
        return (dn, dz) if lab[0] == "L" else (-dn, -dz)

    W = []
    for j in range(K):
        d = {}
        for src in (fixed[j], coef_entries[j]):
            for (a, b), m in src.items():
                key = (index[j][a], index[j + 1][b])
                d[key] = d.get(key, 0.0) + m
        W.append({k: m for k, m in d.items() if np.any(m)})
    return {"channels": chans, "dq": [[shift(l) for l in c] for c in chans], "W": W, "n_sites": K}
