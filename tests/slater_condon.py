"""Matrix elements <D'|H|D> between occupation-number states by the Slater-Condon rules.

A test-side reference, independent of any MPO: the textbook rules for a one- plus two-body
Hamiltonian, written in spin orbitals p = 2 i + s (s = 0 up, 1 down) with the conventions of
the oracle's Fock space (a state is the bit mask of occupied spin orbitals and stands for
prod_{p ascending} a+_p |vac>):

  H = sum_pq h_pq a+_p a_q + 1/2 sum_pqrs <pq|rs> a+_p a+_q a_s a_r + e_const,
  h_pq = h[i_p, i_q] d(s_p, s_q),   <pq|rs> = (i_p i_r | i_q i_s) d(s_p, s_r) d(s_q, s_s),

with chemists' integrals (ij|kl) and the on-site term u_i n_up n_dn written as (ii|ii) = u_i.
  diagonal:            sum_{p occ} h_pp + 1/2 sum_{p,q occ} (<pq|pq> - <pq|qp>) + e_const
  D' = a+_r a_p D:     sign * (h_rp + sum_{q occ in D} (<rq|pq> - <rq|qp>))
  D' = a+_r a+_s a_q a_p D (p < q, r < s):  sign * (<rs|pq> - <rs|qp>)
  more than two spin orbitals apart: 0,
where sign is the fermionic sign of the operator string acting on the bit mask.
"""
from __future__ import annotations

import numpy as np


def _phase(state: int, p: int) -> int:
    return -1 if bin(state & ((1 << p) - 1)).count("1") % 2 else 1


def _apply(state: int, p: int, create: bool):
    """(sign, new state) of a+_p (create) or a_p on a bit mask; sign 0 if it vanishes."""
    occ = (state >> p) & 1
    if occ == (1 if create else 0):
        return 0, state
    return _phase(state, p), state ^ (1 << p)


class SlaterCondon:
    def __init__(self, spec: dict):
        n = spec["n_orb"]
        self.n = n
        self.h = np.asarray(spec["h"], dtype=np.float64)
        eri = np.zeros((n, n, n, n)) if spec.get("eri") is None else np.array(spec["eri"], dtype=np.float64)
        if spec.get("u") is not None:
            for i in range(n):
                eri[i, i, i, i] += spec["u"][i]
        self.eri = eri
        self.e_const = float(spec.get("e_const", 0.0))

    def h1(self, p, q):
        return self.h[p // 2, q // 2] if p % 2 == q % 2 else 0.0

    def g(self, p, q, r, s):
        """<pq|rs>"""
        if p % 2 != r % 2 or q % 2 != s % 2:
            return 0.0
        return self.eri[p // 2, r // 2, q // 2, s // 2]

    def element(self, bra: int, ket: int) -> float:
        occ = [p for p in range(2 * self.n) if (ket >> p) & 1]
        gone = [p for p in occ if not (bra >> p) & 1]            # annihilated (in ket, not in bra)
        new = [p for p in range(2 * self.n) if (bra >> p) & 1 and not (ket >> p) & 1]  # created
        if len(gone) != len(new):
            return 0.0
        if not gone:
            e = sum(self.h1(p, p) for p in occ) + self.e_const
            e += 0.5 * sum(self.g(p, q, p, q) - self.g(p, q, q, p) for p in occ for q in occ)
            return e
        if len(gone) == 1:
            p, r = gone[0], new[0]
            s1, st = _apply(ket, p, False)
            s2, st = _apply(st, r, True)
            assert st == bra
            v = self.h1(r, p) + sum(self.g(r, q, p, q) - self.g(r, q, q, p) for q in occ)
            return s1 * s2 * v
        if len(gone) == 2:
            p, q = gone
            r, s = new
            sign, st = 1, ket
            for orb, create in ((p, False), (q, False), (s, True), (r, True)):  # a+_r a+_s a_q a_p
                f, st = _apply(st, orb, create)
                sign *= f
            assert st == bra
            return sign * (self.g(r, s, p, q) - self.g(r, s, q, p))
        return 0.0


def local_index(state: int, site: int) -> int:
    """Index of the local state of orbital `site` in |0>, |up>, |dn>, |updn>."""
    return ((state >> (2 * site)) & 1) + 2 * ((state >> (2 * site + 1)) & 1)


def sample_pairs(n_orb: int, n_elec: int, two_sz: int, n_states: int, seed: int):
    """Seeded (bra, ket) pairs in the (N, 2Sz) sector: for random kets, the ket itself, random
    single and double excitations that conserve both spins, and a triple excitation."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n_up, n_dn = (n_elec + two_sz) // 2, (n_elec - two_sz) // 2
    pairs = []
    for _ in range(n_states):
        ups = rng.choice(n_orb, n_up, replace=False)
        dns = rng.choice(n_orb, n_dn, replace=False)
        ket = sum(1 << (2 * int(i)) for i in ups) | sum(1 << (2 * int(i) + 1) for i in dns)
        pairs.append((ket, ket))

        def excite(state, k):
            for _ in range(k):
                spin = int(rng.integers(2))
                occ = [p for p in range(spin, 2 * n_orb, 2) if (state >> p) & 1]
                emp = [p for p in range(spin, 2 * n_orb, 2) if not (state >> p) & 1]
                if not occ or not emp:
                    continue
                state ^= (1 << int(rng.choice(occ))) | (1 << int(rng.choice(emp)))
            return state

        for k in (1, 1, 2, 2, 2, 3):
            pairs.append((excite(ket, k), ket))
    return pairs
