"""Pins of the oracle's sweep step (split, truncation, advance, local solve) against facts
fixed outside it, in the full Fock space of small systems:

* with nothing truncated, the state represented by the two-site tensor x at (l, l+1) and
  the one represented by the next guess at (l+1, l+2) of the advanced MPS are the same
  vector of the Fock space (the SVD factorisation is exact);
* with truncation, the state error equals the sum of the discarded squared singular values
  and is orthogonal to the kept state (Eckart-Young for an isometric embedding);
* the new left site tensor is left-canonical;
* the local solve's J* equals -b^T (H_eff - E0)^{-1} b with H_eff = P^T H P built from the
  Fock-space Hamiltonian (independent of the block-sparse environments).
"""
import numpy as np
import pytest

from oracle import blocksparse as BS
from oracle import fock
from oracle import mpo as OM
from oracle import sweep as OW
from workloads import hamiltonians as H
from workloads import mps as M


def _fock_state(mps, vec: dict):
    blocks = M.two_site_blocks(mps)
    tmpl = BS.two_site_template(mps, blocks)
    full = {k: vec.get(k, np.zeros_like(v)) for k, v in tmpl.items()}
    basis = fock.sector_basis(mps["n_sites"], mps["n_elec"], mps["two_sz"])
    P = fock.two_site_isometry(mps, basis, blocks)
    return P @ BS.flatten(full, blocks)


def _case(seed, m=10, center=2):
    spec = H.hubbard_chain(6, t=1.0, U=3.0, n_elec=6)
    mps = M.random_mps(6, 6, 0, m, seed, center=center)
    return spec, mps


@pytest.mark.parametrize("seed,center", [(31, 1), (32, 2), (33, 3)])
def test_exact_split_preserves_state(seed, center):
    spec, mps = _case(seed, center=center)
    x = M.random_two_site_vector(mps, seed + 100)
    before = _fock_state(mps, x)
    site_blocks, new_bond, guess, sv = OW.split(x, mps, 10 ** 6)
    nxt = OW.advance(mps, site_blocks, new_bond)
    after = _fock_state(nxt, guess)
    assert np.linalg.norm(after - before) <= 1e-12 * np.linalg.norm(before)
    assert abs(np.sum(sv ** 2) - np.linalg.norm(before) ** 2) <= 1e-12 * np.linalg.norm(before) ** 2
    assert BS.check_left_canonical(nxt) <= 1e-12


@pytest.mark.parametrize("m_max", [1, 3, 7])
def test_truncation_error_is_discarded_weight(m_max):
    spec, mps = _case(41, m=12, center=2)
    x = M.random_two_site_vector(mps, 141)
    before = _fock_state(mps, x)
    site_blocks, new_bond, guess, sv = OW.split(x, mps, m_max)
    assert sum(d for _, _, d in new_bond) == min(m_max, int(np.count_nonzero(sv)))
    nxt = OW.advance(mps, site_blocks, new_bond)
    after = _fock_state(nxt, guess)
    err = before - after
    assert abs(err @ err - np.sum(sv[m_max:] ** 2)) <= 1e-12 * (before @ before)
    assert abs(err @ after) <= 1e-12 * (before @ before)
    assert BS.check_left_canonical(nxt) <= 1e-12


def test_local_solve_matches_dense_fock():
    spec, mps = _case(51, m=10, center=2)
    blocks = M.two_site_blocks(mps)
    heff = fock.effective_hamiltonian(spec, mps, blocks)
    e0 = float(np.linalg.eigvalsh(heff)[0]) - 0.7
    b = M.random_two_site_vector(mps, 151)
    tmpl = BS.two_site_template(mps, blocks)
    bf = BS.flatten({k: b.get(k, np.zeros_like(v)) for k, v in tmpl.items()}, blocks)
    x, jstar, _ = OW.local_solve(spec, mps, OM.build_mpo(spec), b, e0)
    xd = np.linalg.solve(heff - e0 * np.eye(heff.shape[0]), bf)
    assert abs(jstar - (-bf @ xd)) <= 1e-11 * abs(bf @ xd)
    assert np.linalg.norm(BS.flatten(x, blocks) - xd) <= 1e-10 * np.linalg.norm(xd)
