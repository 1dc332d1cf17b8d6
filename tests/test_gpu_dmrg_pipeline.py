"""Two-site DMRG on the device (lcc.dmrg_sweeps: lcc_sweep, lcc_lowest_eigenpair, lcc_sweep_advance /
_retreat, lcc_sweep_split_block, lcc_sweep_bond, lcc_sweep_site_tensor) and the MPS-LCC pipeline
built on it: the DMRG state of H0 is the reference of the first-order sweep.  Oracle: exact
diagonalisation of H0 and the Fock-space first-order theory (oracle/perturbation.py), on the
ab initio system of 6 orbitals with the Fink partition (core 0-1, active 2-3, virtual 4-5).

* Full bond dimension: the DMRG energy equals the lowest eigenvalue of H0 and the read-out MPS
  is its eigenvector (Fock-space contraction of the exported tensors); E2 and E3 from the
  pipeline equal the oracle's.
* Truncated DMRG (M = 6): the energy is a variational upper bound, the read-out MPS is a
  normalised state whose H0 expectation is that energy, and the projector-approximation sweep on
  it reproduces the oracle's first-order theory for that reference.
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


def test_dmrg_then_first_order(system):
    torch, lcc = need_gpu()
    spec, s0, su, basis, h0, u, h = system
    w, V = np.linalg.eigh(h0)
    ref = PT.first_order(h0, u, u, V[:, 0])
    ctx = lcc.Context(0)
    H0, U = lcc.create_hamiltonian(ctx, s0), lcc.create_hamiltonian(ctx, su)
    d = lcc.dmrg_sweeps(ctx, H0, M.random_mps(K, N, SZ, 400, seed=31, center=0), m_max=400, sweeps=2)
    phi = fock.mps_state(d["mps"], basis)
    ov = abs(float(phi @ V[:, 0]))
    say(f"[dmrg] E {d['energy']:.12f} (exact {w[0]:.12f}), |<phi|phi0>| {ov:.12f}, |phi| {np.linalg.norm(phi):.12f}")
    assert abs(d["energy"] - w[0]) <= 1e-10 * abs(w[0])
    assert abs(np.linalg.norm(phi) - 1.0) <= 1e-10
    assert abs(ov - 1.0) <= 1e-9
    psi0 = d["mps"]
    site = psi0["center"]
    e0 = lcc.mps_expectation(ctx, H0, psi0, site)
    e1 = lcc.mps_expectation(ctx, U, psi0, site)
    assert abs(e0 - w[0]) <= 1e-10 * abs(w[0])
    out = lcc.first_order_sweeps(ctx, H0, U, M.random_mps(K, N, SZ, 400, seed=32, center=0), psi0, e0=e0, c=e1,
                                 m_max=400, sweeps=2, u=U, e1=e1)
    say(f"[dmrg] pipeline E2 {out['e2']:.12f} (oracle {ref['e2']:.12f}), E3 {out['e3']:.12f} (oracle {ref['e3']:.12f})")
    assert abs(out["e2"] - ref["e2"]) <= 1e-8 * abs(ref["e2"])
    assert abs(out["e3"] - ref["e3"]) <= 1e-7 * max(abs(ref["e3"]), abs(ref["e2"]))


def test_truncated_dmrg_reference(system):
    torch, lcc = need_gpu()
    spec, s0, su, basis, h0, u, h = system
    w = np.linalg.eigvalsh(h0)
    ctx = lcc.Context(0)
    H0, U, Hf = (lcc.create_hamiltonian(ctx, s0), lcc.create_hamiltonian(ctx, su), lcc.create_hamiltonian(ctx, spec))
    d = lcc.dmrg_sweeps(ctx, H0, M.random_mps(K, N, SZ, 6, seed=33, center=0), m_max=6, sweeps=3)
    phi = fock.mps_state(d["mps"], basis)
    say(f"[dmrg] M=6: E {d['energy']:.10f} (exact {w[0]:.10f}), <phi|H0|phi> {float(phi @ h0 @ phi):.10f}")
    assert d["energy"] >= w[0] - 1e-10 * abs(w[0])
    assert abs(np.linalg.norm(phi) - 1.0) <= 1e-10
    assert abs(float(phi @ h0 @ phi) - d["energy"]) <= 1e-9 * abs(w[0])
    ref = PT.first_order(h0, h, u, phi)
    if ref["lambda_min"] <= 1e-6:
        pytest.skip("the truncated reference leaves Q(H0 - E0)Q indefinite")
    psi0 = d["mps"]
    site = psi0["center"]
    e0 = lcc.mps_expectation(ctx, H0, psi0, site)
    c = lcc.mps_expectation(ctx, Hf, psi0, site)
    e1 = lcc.mps_expectation(ctx, U, psi0, site)
    assert abs(e0 - ref["e0"]) <= 1e-10 * abs(ref["e0"])
    assert abs(c - ref["c"]) <= 1e-10 * abs(ref["c"])
    out = lcc.first_order_sweeps(ctx, H0, Hf, M.random_mps(K, N, SZ, 400, seed=34, center=0), psi0, e0=e0, c=c,
                                 m_max=400, sweeps=2, u=U, e1=e1)
    say(f"[dmrg] projector approximation on the M=6 reference: E2 {out['e2']:.12f} (oracle {ref['e2']:.12f})")
    assert abs(out["e2"] - ref["e2"]) <= 1e-8 * abs(ref["e2"])
    assert abs(out["e3"] - ref["e3"]) <= 1e-7 * max(abs(ref["e3"]), abs(ref["e2"]))
