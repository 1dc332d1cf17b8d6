"""Pins of the oracle's first-order vectors (oracle.fock.first_order_vectors): with the bra equal
to the ket the overlap vector is the ket's own two-site tensor and u is H_eff applied to it;
with complete bases on both sides the isometry is unitary on the sector, so the local vectors
keep the norms of Phi0 and H Phi0 (Parseval)."""
import numpy as np

from oracle import blocksparse as BS
from oracle import fock
from workloads import hamiltonians as H
from workloads import mps as M


def two_site_tensor(mps, l):
    """x[a, s1, s2, b] = sum_c A_l^{s1}[a, c] A_{l+1}^{s2}[c, b] (input assembly for the pins)."""
    out = {}
    right = {}
    for il, s, ir, a in mps["sites"][l + 1]:
        right.setdefault(il, []).append((s, ir, a))
    for il, s1, ic, a1 in mps["sites"][l]:
        for s2, ib, a2 in right.get(ic, []):
            key = (il, s1, s2, ib)
            out[key] = out.get(key, 0.0) + a1 @ a2
    return out


def test_bra_equal_to_ket():
    spec = H.random_ab_initio(6, 5, two_sz=1, seed=9)
    mps = M.random_mps(6, 5, 1, 12, seed=10, center=2)
    blocks = M.two_site_blocks(mps)
    tmpl = BS.two_site_template(mps, blocks)
    x0 = BS.flatten({k: two_site_tensor(mps, 2).get(k, np.zeros_like(v)) for k, v in tmpl.items()}, blocks)
    u, v, e1 = fock.first_order_vectors(spec, mps, mps, blocks)
    heff = fock.effective_hamiltonian(spec, mps, blocks)
    assert np.abs(v - x0).max() <= 1e-13 * np.abs(x0).max()
    assert np.linalg.norm(u - heff @ x0) <= 1e-12 * np.linalg.norm(u)
    assert abs(e1 - x0 @ heff @ x0 / (x0 @ x0)) <= 1e-12 * abs(e1)


def test_complete_bases_keep_norms():
    spec = H.hubbard_chain(6, U=3.0, n_elec=6)
    bra = M.random_mps(6, 6, 0, 64, seed=11, center=2)   # complete at every bond
    ket = M.random_mps(6, 6, 0, 4, seed=12, center=4)    # truncated, other gauge
    blocks = M.two_site_blocks(bra)
    u, v, e1 = fock.first_order_vectors(spec, bra, ket, blocks)
    basis = fock.sector_basis(6, 6, 0)
    phi0 = fock.mps_state(ket, basis)
    hphi = fock.hamiltonian_matrix(spec, basis) @ phi0
    assert abs(np.linalg.norm(v) - np.linalg.norm(phi0)) <= 1e-12 * np.linalg.norm(phi0)
    assert abs(np.linalg.norm(u) - np.linalg.norm(hphi)) <= 1e-12 * np.linalg.norm(hphi)
    # the ket state from the contraction of its two-site tensor with its own isometry
    kb = M.two_site_blocks(ket)
    kt = BS.two_site_template(ket, kb)
    x0 = BS.flatten({k: two_site_tensor(ket, 4).get(k, np.zeros_like(t)) for k, t in kt.items()}, kb)
    assert np.linalg.norm(fock.two_site_isometry(ket, basis, kb) @ x0 - phi0) <= 1e-13 * np.linalg.norm(phi0)
