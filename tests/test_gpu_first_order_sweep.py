"""The first-order MPS-LCC sweep on the device (lcc.first_order_sweeps: lcc_sweep with a reference
MPS attached, lcc_sweep_first_order_rhs, lcc_solve_local_lcc, lcc_sweep_advance / _retreat,
lcc_sweep_u_expectation, lcc_mps_expectation) against the oracle's Fock-space first-order
theory (oracle/perturbation.py), on an ab initio system of 6 orbitals with the Fink partition
(core 0-1, active 2-3, virtual 4-5).

* Full bond dimension: from the second block on the two-site space spans the sector (the
  first block's right basis is the random initial MPS's, a 16-dimensional part of the space
  of sites 2-5), so every later local solve is exact; E0, E1 from the MPS expectations, E2 (the
  Hylleraas values) and E3 match the oracle to ~1e-9, over two sweeps (right, then left: both
  split directions), and the first value is an upper bound.
* Truncated bond dimension: every Hylleraas value is an upper bound of the exact E2.
* Projector approximation (O = H, an approximate reference): E0 = <Phi0|H0|Phi0>,
  c = <Phi0|H|Phi0>, E2 = <Phi0|H|Phi1> and E3 against the oracle.
"""
import numpy as np
import pytest

from gpu_common import need_gpu, say
from oracle import fock
from oracle import perturbation as PT
from workloads import hamiltonians as H
from workloads import mps as M

pytestmark = pytest.mark.gpu
CLASSES = np.array([0, 0, 1, 1, 2, 2], dtype=np.int32)
K, N, SZ = 6, 6, 0


@pytest.fixture(scope="module")
def system():
    spec = dict(H.random_ab_initio(K, N, two_sz=SZ, seed=11), e_const=0.3)
    basis = fock.sector_basis(K, N, SZ)
    s0, su = H.with_partition(spec, CLASSES, 1), H.with_partition(spec, CLASSES, 2)
    h0 = fock.hamiltonian_matrix(s0, basis).toarray()
    u = fock.hamiltonian_matrix(su, basis).toarray()
    h = fock.hamiltonian_matrix(spec, basis).toarray()
    return spec, s0, su, basis, h0, u, h


def _mps_of(vec, basis):
    full = np.zeros(4 ** K)
    full[fock.config_index(basis, K)] = vec / np.linalg.norm(vec)
    return M.mps_from_amplitudes(full, K, N, SZ)


def _hams(lcc, ctx, spec, s0, su):
    return (lcc.create_hamiltonian(ctx, s0), lcc.create_hamiltonian(ctx, su), lcc.create_hamiltonian(ctx, spec))


def test_full_bond_dimension_is_exact(system):
    torch, lcc = need_gpu()
    spec, s0, su, basis, h0, u, h = system
    phi0 = PT.rayleigh_schrodinger(h0, u)["phi0"]
    ref = PT.first_order(h0, u, u, phi0)
    ctx = lcc.Context(0)
    H0, U, _ = _hams(lcc, ctx, spec, s0, su)
    psi0 = _mps_of(phi0, basis)
    e0 = lcc.mps_expectation(ctx, H0, psi0, 0)
    e1 = lcc.mps_expectation(ctx, U, psi0, 0)
    say(f"[first-order] E0 {e0:.12f} (oracle {ref['e0']:.12f}), E1 {e1:.3e}")
    assert abs(e0 - ref["e0"]) <= 1e-11 * abs(ref["e0"])
    assert abs(e1 - ref["e1"]) <= 1e-11
    psi1 = M.random_mps(K, N, SZ, 400, seed=21, center=0)
    out = lcc.first_order_sweeps(ctx, H0, U, psi1, psi0, e0=e0, c=e1, m_max=400, sweeps=2, u=U, e1=e1)
    say(f"[first-order] E2 {out['e2']:.12f} (oracle {ref['e2']:.12f}), E3 {out['e3']:.12f} "
        f"(oracle {ref['e3']:.12f}), {len(out['hylleraas'])} local solves")
    say(f"[first-order] local values {[round(v, 9) for v in out['hylleraas']]} blocks {out['blocks']}")
    scale = abs(ref["e2"])
    assert len(out["hylleraas"]) == 2 * (K - 1) - 1
    assert out["hylleraas"][0] >= ref["e2"] - 1e-9 * scale
    for j in out["hylleraas"][1:]:
        assert abs(j - ref["e2"]) <= 1e-9 * scale
    assert abs(out["e3"] - ref["e3"]) <= 1e-8 * max(abs(ref["e3"]), scale)
    assert abs(out["norm2"] - float(ref["phi1"] @ ref["phi1"])) <= 1e-8 * float(ref["phi1"] @ ref["phi1"])


def test_truncated_sweeps_bound_e2(system):
    torch, lcc = need_gpu()
    spec, s0, su, basis, h0, u, h = system
    phi0 = PT.rayleigh_schrodinger(h0, u)["phi0"]
    ref = PT.first_order(h0, u, u, phi0)
    ctx = lcc.Context(0)
    H0, U, _ = _hams(lcc, ctx, spec, s0, su)
    psi0 = _mps_of(phi0, basis)
    e0 = lcc.mps_expectation(ctx, H0, psi0, 0)
    psi1 = M.random_mps(K, N, SZ, 6, seed=22, center=0)
    out = lcc.first_order_sweeps(ctx, H0, U, psi1, psi0, e0=e0, c=0.0, m_max=6, sweeps=3)
    say(f"[first-order] m=6: J {out['hylleraas'][0]:.9f} .. {out['hylleraas'][-1]:.9f} (exact E2 {ref['e2']:.9f})")
    for j in out["hylleraas"]:
        assert j >= ref["e2"] - 1e-9 * abs(ref["e2"])
    assert out["hylleraas"][-1] <= out["hylleraas"][0] + 1e-9 * abs(ref["e2"])


def test_projector_approximation(system):
    torch, lcc = need_gpu()
    spec, s0, su, basis, h0, u, h = system
    phi0 = PT.rayleigh_schrodinger(h0, u)["phi0"]
    rng = np.random.default_rng(5)
    # an approximate reference inside the ground state's class occupations
    occ = np.zeros((basis.size, 3), dtype=np.int64)
    for p, c in enumerate(CLASSES):
        occ[:, c] += ((basis >> (2 * p)) & 1) + ((basis >> (2 * p + 1)) & 1)
    same = (occ == occ[int(np.argmax(np.abs(phi0)))]).all(axis=1)
    phi = phi0 + 0.05 * rng.standard_normal(basis.size) * same
    phi /= np.linalg.norm(phi)
    ref = PT.first_order(h0, h, u, phi)
    assert ref["lambda_min"] > 0
    ctx = lcc.Context(0)
    H0, U, Hf = _hams(lcc, ctx, spec, s0, su)
    psi0 = _mps_of(phi, basis)
    e0 = lcc.mps_expectation(ctx, H0, psi0, 0)
    c = lcc.mps_expectation(ctx, Hf, psi0, 0)
    e1 = lcc.mps_expectation(ctx, U, psi0, 0)
    assert abs(e0 - ref["e0"]) <= 1e-11 * abs(ref["e0"])
    assert abs(c - ref["c"]) <= 1e-11 * abs(ref["c"])
    psi1 = M.random_mps(K, N, SZ, 400, seed=23, center=0)
    out = lcc.first_order_sweeps(ctx, H0, Hf, psi1, psi0, e0=e0, c=c, m_max=400, sweeps=2, u=U, e1=e1)
    say(f"[first-order] projector approximation: E2 {out['e2']:.12f} (oracle {ref['e2']:.12f}), "
        f"E3 {out['e3']:.12f} (oracle {ref['e3']:.12f})")
    scale = abs(ref["e2"])
    assert abs(out["e2"] - ref["e2"]) <= 1e-9 * scale
    assert abs(out["e3"] - ref["e3"]) <= 1e-8 * max(abs(ref["e3"]), scale)
