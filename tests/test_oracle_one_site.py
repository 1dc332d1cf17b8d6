"""Pins of the oracle's one-site local problem (Implementation section, local-derivative figure:
the derivative with respect to one site tensor A^{n_l}, 4 M^2 unknowns) --
oracle.fock.one_site_isometry / effective_hamiltonian_one_site and
oracle.blocksparse.one_site_apply:

* P1 is an isometry when the sites left of the center are left-canonical and those right of it
  right-canonical (P1^T P1 = 1);
* the one-site basis is the two-site basis of (c, c+1) times the fixed right-canonical site
  c+1 (P1 = P2 E), so H1 = E^T H2 E with the two-site H_eff pinned elsewhere;
* an exact eigenstate: the MPS of the ground state of H, brought into the one-site gauge at
  any site l, has its site tensor as an eigenvector of H1 with eigenvalue E0, which is the
  lowest eigenvalue of H1 (the one-site space contains the ground state);
* the block-sparse route (one_site_apply) equals the dense H1 on truncated bases.
"""
import numpy as np
import pytest

from oracle import blocksparse as BS
from oracle import fock
from oracle import mpo as OM
from workloads import hamiltonians as H
from workloads import mps as M

SYSTEMS = {
    "abinitio_k6_m10": lambda: (H.random_ab_initio(6, 6, seed=21), M.random_mps(6, 6, 0, 10, seed=22, center=2)),
    "hubbard_4x2_m16": lambda: (H.hubbard_2d(4, 2, U=4.0, n_elec=7, two_sz=1),
                                M.random_mps(8, 7, 1, 16, seed=8, center=3)),
}


def _flat(vec, keys):
    return np.concatenate([vec[k].reshape(-1) for k in keys])


@pytest.mark.parametrize("name", sorted(SYSTEMS))
@pytest.mark.parametrize("site", [0, 2, 4])
def test_isometry_and_two_site_relation(name, site):
    spec, mps = SYSTEMS[name]()
    m1 = M.canonical_at(mps, site)
    basis = fock.sector_basis(spec["n_orb"], spec["n_elec"], spec["two_sz"])
    keys1 = [(a, s, 0, b) for a, s, b in M.one_site_blocks(m1)]
    P1 = fock.one_site_isometry(m1, basis, keys1)
    assert np.abs(P1.T @ P1 - np.eye(P1.shape[1])).max() <= 1e-12
    keys2 = M.two_site_blocks(m1)
    P2 = fock.two_site_isometry(m1, basis, keys2)
    # E column by column: the two-site tensor of each one-site unit vector
    n1 = P1.shape[1]
    E = np.zeros((P2.shape[1], n1))
    shapes = {k: (m1["bonds"][site][k[0]][2], m1["bonds"][site + 1][k[3]][2]) for k in keys1}
    col = 0
    for k in keys1:
        r, c = shapes[k]
        for i in range(r):
            for j in range(c):
                x1 = {kk: np.zeros(shapes[kk]) for kk in keys1}
                x1[k][i, j] = 1.0
                E[:, col] = _flat(BS.one_site_embed(m1, x1, keys2), keys2)
                col += 1
    assert np.abs(P2 @ E - P1).max() <= 1e-12
    H1 = fock.effective_hamiltonian_one_site(spec, m1, keys1)
    H2 = fock.effective_hamiltonian(spec, m1, keys2)
    assert np.abs(E.T @ H2 @ E - H1).max() <= 1e-11 * np.abs(H1).max()


@pytest.mark.parametrize("site", [0, 1, 3, 5])
def test_exact_eigenstate_site_tensor_is_an_eigenvector(site):
    spec = dict(H.random_ab_initio(6, 6, two_sz=0, seed=11), e_const=0.3)
    basis = fock.sector_basis(6, 6, 0)
    w, V = np.linalg.eigh(fock.hamiltonian_matrix(spec, basis).toarray())
    full = np.zeros(4 ** 6)
    full[fock.config_index(basis, 6)] = V[:, 0]
    m1 = M.canonical_at(M.mps_from_amplitudes(full, 6, 6, 0), site)
    keys1 = [(a, s, 0, b) for a, s, b in M.one_site_blocks(m1)]
    H1 = fock.effective_hamiltonian_one_site(spec, m1, keys1)
    # the site tensor in the layout of the keys
    blocks = {(il, s, 0, ir): A for il, s, ir, A in m1["sites"][site]}
    a = np.concatenate([blocks[k].reshape(-1) if k in blocks else
                        np.zeros(m1["bonds"][site][k[0]][2] * m1["bonds"][site + 1][k[3]][2]) for k in keys1])
    assert abs(np.linalg.norm(a) - 1.0) <= 1e-12
    assert np.abs(H1 @ a - w[0] * a).max() <= 1e-11 * abs(w[0])
    assert abs(np.linalg.eigvalsh(H1)[0] - w[0]) <= 1e-11 * abs(w[0])


@pytest.mark.parametrize("name", sorted(SYSTEMS))
def test_blocksparse_route_equals_dense(name):
    spec, mps = SYSTEMS[name]()
    site = mps["center"]
    m1 = M.canonical_at(mps, site)
    keys1 = [(a, s, 0, b) for a, s, b in M.one_site_blocks(m1)]
    x = M.random_one_site_vector(m1, 5)
    y = BS.one_site_apply(spec, m1, OM.build_mpo(spec), x)
    H1 = fock.effective_hamiltonian_one_site(spec, m1, keys1)
    yd = H1 @ _flat(x, keys1)
    assert np.abs(_flat(y, keys1) - yd).max() <= 1e-12 * np.abs(yd).max()
