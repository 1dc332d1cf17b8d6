"""Pins of the first-order oracle (oracle/perturbation.py) against what the mathematics fixes:

* the linear-solve route (first-order equation, Wigner 2n+1 energies) equals the textbook
  spectral sums of RS perturbation theory over the eigenstates of H0;
* E1, E2, E3 are the Taylor coefficients of the lowest eigenvalue of H0 + lambda U at lambda = 0
  (a polynomial fit of exact eigenvalues, a third route);
* for an exact eigenstate of H0 the projector approximation (O = H) gives the same Phi1, E2, E3
  as O = U;
* the Hylleraas functional is an upper bound of E2 on the complement of Phi0 and equals it at
  Phi1;
* the MPS built from a state's amplitudes (the input helper of the first-order tests)
  contracts back to that state.
"""
import numpy as np
import pytest

from oracle import fock
from oracle import perturbation as PT
from workloads import hamiltonians as H
from workloads import mps as M

CLASSES = np.array([0, 0, 1, 1, 2, 2], dtype=np.int32)


def _parts(spec, classes):
    basis = fock.sector_basis(spec["n_orb"], spec["n_elec"], spec["two_sz"])
    h0 = fock.hamiltonian_matrix(H.with_partition(spec, classes, 1), basis).toarray()
    u = fock.hamiltonian_matrix(H.with_partition(spec, classes, 2), basis).toarray()
    h = fock.hamiltonian_matrix(spec, basis).toarray()
    return basis, h0, u, h


SYSTEMS = [
    lambda: (dict(H.random_ab_initio(6, 6, two_sz=0, seed=11), e_const=0.3), CLASSES),
    lambda: (H.random_ab_initio(5, 5, two_sz=1, seed=12), np.array([0, 1, 1, 1, 2], dtype=np.int32)),
]


@pytest.mark.parametrize("make", SYSTEMS)
def test_linear_solve_equals_spectral_sums(make):
    spec, cls = make()
    _, h0, u, _ = _parts(spec, cls)
    rs = PT.rayleigh_schrodinger(h0, u)
    fo = PT.first_order(h0, u, u, rs["phi0"])
    scale = abs(rs["e2"]) + abs(rs["e3"])
    assert abs(fo["e0"] - rs["e0"]) <= 1e-12 * abs(rs["e0"])
    assert abs(fo["e1"] - rs["e1"]) <= 1e-12 * scale
    assert abs(fo["e2"] - rs["e2"]) <= 1e-11 * scale
    assert abs(fo["e3"] - rs["e3"]) <= 1e-11 * scale
    assert fo["lambda_min"] > 0  # Phi0 is the ground state: the first-order operator is positive
    # the Fink partition: U moves electrons between classes, so <Phi0|U|Phi0> = 0
    assert abs(rs["e1"]) <= 1e-12 * scale


def test_energies_are_taylor_coefficients():
    spec, cls = SYSTEMS[0]()
    _, h0, u, _ = _parts(spec, cls)
    fo = PT.first_order(h0, u, u, PT.rayleigh_schrodinger(h0, u)["phi0"])
    lam = np.linspace(-0.05, 0.05, 41)
    e = np.array([np.linalg.eigvalsh(h0 + x * u)[0] for x in lam])
    c = np.polynomial.polynomial.polyfit(lam, e, 10)
    assert abs(c[0] - fo["e0"]) <= 1e-9 * abs(fo["e0"])
    assert abs(c[1] - fo["e1"]) <= 1e-8
    assert abs(c[2] - fo["e2"]) <= 1e-6 * abs(fo["e2"])
    assert abs(c[3] - fo["e3"]) <= 1e-4 * abs(fo["e3"])


def test_projector_approximation_reduces_for_an_exact_reference():
    spec, cls = SYSTEMS[0]()
    _, h0, u, h = _parts(spec, cls)
    phi0 = PT.rayleigh_schrodinger(h0, u)["phi0"]
    a = PT.first_order(h0, u, u, phi0)
    b = PT.first_order(h0, h, u, phi0)
    assert np.abs(a["phi1"] - b["phi1"]).max() <= 1e-10 * np.abs(a["phi1"]).max()
    assert abs(a["e2"] - b["e2"]) <= 1e-11 * abs(a["e2"])
    # an approximate reference: E0 is its H0 expectation, the two right-hand sides now differ
    rng = np.random.default_rng(3)
    phi = phi0 + 0.05 * rng.standard_normal(phi0.size)
    phi /= np.linalg.norm(phi)
    c = PT.first_order(h0, h, u, phi)
    assert abs(c["e0"] - float(phi @ h0 @ phi)) <= 1e-12 * abs(c["e0"])
    assert abs(float(phi @ c["phi1"])) <= 1e-12
    assert abs(c["e2"] - PT.first_order(h0, u, u, phi)["e2"]) > 1e-6


def test_hylleraas_bound():
    spec, cls = SYSTEMS[1]()
    _, h0, u, _ = _parts(spec, cls)
    phi0 = PT.rayleigh_schrodinger(h0, u)["phi0"]
    fo = PT.first_order(h0, u, u, phi0)
    assert abs(PT.hylleraas(h0, u, phi0, fo["phi1"]) - fo["e2"]) <= 1e-11 * abs(fo["e2"])
    rng = np.random.default_rng(4)
    for _ in range(20):
        z = fo["phi1"] + 0.3 * rng.standard_normal(phi0.size) * np.abs(fo["phi1"]).max()
        z -= phi0 * float(phi0 @ z)
        assert PT.hylleraas(h0, u, phi0, z) >= fo["e2"] - 1e-12


@pytest.mark.parametrize("K,N,sz,seed", [(5, 4, 0, 3), (6, 5, 1, 4), (6, 6, 0, 5)])
def test_mps_from_amplitudes_round_trip(K, N, sz, seed):
    basis = fock.sector_basis(K, N, sz)
    rng = np.random.default_rng(seed)
    psi = rng.standard_normal(basis.size)
    psi /= np.linalg.norm(psi)
    full = np.zeros(4 ** K)
    full[fock.config_index(basis, K)] = psi
    m = M.mps_from_amplitudes(full, K, N, sz)
    assert np.abs(fock.mps_state(m, basis) - psi).max() <= 1e-13
    # right-canonical sites 2..K-1
    for j in range(2, K):
        dl = [d for _, _, d in m["bonds"][j]]
        for il in range(len(dl)):
            blks = [b for b in m["sites"][j] if b[0] == il]
            g = sum(b[3] @ b[3].T for b in blks)
            assert np.abs(g - np.eye(dl[il])).max() <= 1e-12
