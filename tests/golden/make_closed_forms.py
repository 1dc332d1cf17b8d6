"""Writes closed_forms.json: textbook closed forms used as oracle pins (no oracle code).

* Hubbard dimer (two sites, two electrons, Sz = 0): the singlet ground energy is
  (U - sqrt(U^2 + 16 t^2)) / 2.
* Open tight-binding chain of L sites: one-particle levels -2 t cos(k pi / (L + 1)),
  k = 1..L; the U = 0 ground energy at half filling, Sz = 0, fills the lowest L/2 twice.
* Bipartite half-filled Hubbard chain (particle-hole + sublattice symmetry): the spectrum
  in the N = L, Sz = 0 sector is symmetric about U L / 4, so lambda_min + lambda_max = U L / 2,
  and the trace is U * L / 4 * dim (each site is doubly occupied with probability 1/4).
"""
import json
import math
import os

t, U, L = 1.0, 4.0, 8
dim = math.comb(L, L // 2) ** 2
out = {
    "hubbard_dimer_t1_U4_ground": (U - math.sqrt(U * U + 16 * t * t)) / 2,
    "tight_binding_obc_L8_halffilling_ground": 2 * sum(-2 * t * math.cos(k * math.pi / (L + 1)) for k in range(1, L // 2 + 1)),
    "hubbard_chain_L8_U4_lmin_plus_lmax": U * L / 2,
    "hubbard_chain_L8_U4_trace": U * L / 4 * dim,
    "hubbard_chain_L8_sector_dim": dim,
}
with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "closed_forms.json"), "w") as f:
    json.dump(out, f, indent=1, sort_keys=True)
    f.write("\n")
