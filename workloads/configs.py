"""The named synthetic workloads (Hamiltonian + MPS + vectors), seeded.

Shapes follow the paper's benchmark families (Benchmarks section): a 1-D Hubbard chain
(complete basis, exact-diagonalisation check), the 2-D 1-band Hubbard model, a synthetic
ab initio Hamiltonian standing in for the molecular integrals, and the 3-band Cu-O model.
The paper's integrals and lattices are not available, so these stand in for them.
"""
from __future__ import annotations

import numpy as np

from . import hamiltonians as H
from . import mps as M


WORKLOADS = {
    # name: (hamiltonian factory, m_max, seed)
    "hubbard1d_k8_m64": (lambda: H.hubbard_chain(8, t=1.0, U=4.0, n_elec=8, two_sz=0), 64, 1001),
    "hubbard2d_4x4_m500": (lambda: H.hubbard_2d(4, 4, t=1.0, U=4.0, n_elec=14, two_sz=0), 500, 1002),
    "abinitio_k24_m1000": (lambda: H.random_ab_initio(24, 12, two_sz=0, seed=1003), 1000, 1003),
    "threeband_4x2_m2000": (lambda: H.three_band(4, 2, n_holes=9, two_sz=1), 2000, 1004),
}


def free_fermion_energy(h: np.ndarray, n_up: int, n_dn: int) -> float:
    """Ground energy of sum h_ij c+ c for n_up up and n_dn down electrons (the U = 0 bound)."""
    e = np.linalg.eigvalsh(h)
    return float(np.sum(e[:n_up]) + np.sum(e[:n_dn]))


def make(name: str, m_max: int | None = None, seed: int | None = None, center: int | None = None):
    """Return (hamiltonian spec, mps) for a named workload; m_max/seed override the defaults."""
    factory, m_default, seed_default = WORKLOADS[name]
    spec = factory()
    m = m_default if m_max is None else m_max
    sd = seed_default if seed is None else seed
    mps = M.random_mps(spec["n_orb"], spec["n_elec"], spec["two_sz"], m, sd, center=center)
    return spec, mps


def lower_bound_shift(spec: dict, gamma: float = 0.5) -> float:
    """E0 = E(U=0) - gamma for Hamiltonians whose two-body part is a non-negative on-site U.

    Such an H satisfies H >= its one-body part, so by Cauchy interlacing through the MPS
    isometry the lowest eigenvalue of the local effective Hamiltonian is >= E(U=0), and
    H_eff - E0 is positive definite.
    """
    if spec["eri"] is not None or (spec["u"] is not None and np.any(spec["u"] < 0)):
        raise ValueError("lower_bound_shift needs a one-body + non-negative on-site U Hamiltonian")
    n, tsz = spec["n_elec"], spec["two_sz"]
    n_up, n_dn = (n + tsz) // 2, (n - tsz) // 2
    return free_fermion_energy(spec["h"], n_up, n_dn) + spec["e_const"] - gamma


BATCH_PARENTS = ("hubbard2d_4x4_m500", "abinitio_k24_m1000", "threeband_4x2_m2000")


def batch_members(n: int = 64, seed: int = 1005, m_range=(128, 1500), parents=BATCH_PARENTS) -> list:
    """(parent workload, M, seed) of n independent local problems: parents uniform over the
    lattice / ab initio families, M uniform in m_range, per-problem seed = seed*1000 + i."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(n):
        parent = parents[int(rng.integers(len(parents)))]
        m = int(rng.integers(m_range[0], m_range[1] + 1))
        out.append((parent, m, seed * 1000 + i))
    return out


def make_member(parent: str, m_max: int, seed: int, jitter_sigma: float = 0.5):
    """A batch member: the parent's Hamiltonian and an MPS whose bond weights carry a
    lognormal(sigma) jitter per sector, so the block histograms differ between members."""
    factory, _, _ = WORKLOADS[parent]
    spec = factory()
    mps = M.random_mps(spec["n_orb"], spec["n_elec"], spec["two_sz"], m_max, seed, jitter_sigma=jitter_sigma)
    return spec, mps
