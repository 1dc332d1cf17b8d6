"""Plant plausible mistakes in the oracle (CPU only) and check that a pin catches each one."""
import itertools

import numpy as np

from oracle import fock
from oracle import mpo as OM
from workloads import hamiltonians as H


def _mpo_matches_fock(spec):
    mpo = OM.build_mpo(spec)
    D = OM.dense_operator(mpo)
    basis = fock.sector_basis(spec["n_orb"], spec["n_elec"], spec["two_sz"])
    idx = np.zeros(basis.size, dtype=np.int64)
    for j in range(spec["n_orb"]):
        idx = idx * 4 + ((basis >> (2 * j)) & 1) + 2 * ((basis >> (2 * j + 1)) & 1)
    Hs = fock.hamiltonian_matrix(spec, basis).toarray()
    return np.abs(D[np.ix_(idx, idx)] - Hs).max() < 1e-12


def test_wrong_local_sign_is_caught(monkeypatch):
    spec = H.hubbard_chain(3, U=2.0, n_elec=3, two_sz=1)
    assert _mpo_matches_fock(spec)
    bad = OM._CDAG_DN.copy()
    bad[3, 1] = +1.0
    monkeypatch.setattr(OM, "_CDAG_DN", bad)
    assert not _mpo_matches_fock(spec)


def test_missing_jordan_wigner_string_is_caught(monkeypatch):
    spec = H.hubbard_chain(3, U=2.0, n_elec=3, two_sz=1)
    monkeypatch.setattr(OM, "F", np.eye(4))
    assert not _mpo_matches_fock(spec)


def test_two_body_index_swap_is_caught(monkeypatch):
    base = H.hubbard_chain(4, t=1.0, U=3.0, n_elec=4)
    rot = H.rotate_orbitals(base, H.random_orthogonal(4, 11))
    good = fock.operator_strings

    def swapped(spec):
        n = spec["n_orb"]
        eri = spec["eri"]
        if eri is None:
            yield from good(spec)
            return
        for coef, ops in good(dict(spec, eri=None)):
            yield coef, ops
        for i, j, k, l in itertools.product(range(n), repeat=4):
            for s, t in itertools.product((0, 1), repeat=2):
                # a+_i a+_k a_j a_l instead of a+_i a+_k a_l a_j
                yield 0.5 * eri[i, j, k, l], [(2 * i + s, True), (2 * k + t, True), (2 * j + s, False), (2 * l + t, False)]

    monkeypatch.setattr(fock, "operator_strings", swapped)
    w0 = np.linalg.eigvalsh(fock.hamiltonian_matrix(base).toarray())
    w1 = np.linalg.eigvalsh(fock.hamiltonian_matrix(rot).toarray())
    assert np.abs(w0 - w1).max() > 1e-3


def _twosided_matches_fock(spec, switch=None):
    mpo = OM.build_mpo_twosided(spec, switch)
    D = OM.dense_operator(mpo)
    basis = fock.sector_basis(spec["n_orb"], spec["n_elec"], spec["two_sz"])
    idx = np.zeros(basis.size, dtype=np.int64)
    for j in range(spec["n_orb"]):
        idx = idx * 4 + ((basis >> (2 * j)) & 1) + 2 * ((basis >> (2 * j + 1)) & 1)
    Hs = fock.hamiltonian_matrix(spec, basis).toarray()
    return np.abs(D[np.ix_(idx, idx)] - Hs).max() < 1e-12


def test_twosided_mpo_planted_mistakes_are_caught(monkeypatch):
    spec = H.random_ab_initio(4, 3, two_sz=1, seed=13)
    assert _twosided_matches_fock(spec) and _twosided_matches_fock(spec, 1)
    # a pass-through or event without its Jordan-Wigner parity
    with monkeypatch.context() as m:
        m.setattr(OM, "F", np.eye(4))
        assert not _twosided_matches_fock(spec)
    # a wrong local sign of c+_dn |up>
    with monkeypatch.context() as m:
        bad = OM._CDAG_DN.copy()
        bad[3, 1] = +1.0
        m.setattr(OM, "_CDAG_DN", bad)
        assert not _twosided_matches_fock(spec)
    # a dropped permutation sign when the operator string is sorted by site
    with monkeypatch.context() as m:
        good = OM._site_strings
        m.setattr(OM, "_site_strings", lambda s: ((abs(c), ops) for c, ops in good(s)))
        assert not _twosided_matches_fock(spec)
