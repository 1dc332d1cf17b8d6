"""Host-side checks of the C ABI library (no GPU needed).

* the library loads and exports every function declared in include/mpslcc.h;
* the MPO the library compiles contracts to the Fock-space Hamiltonian of the oracle
  (O1) on small systems of every Hamiltonian family, including the two-operator channel
  switch;
* argument errors come back as status codes.
"""
import os
import re

import numpy as np
import pytest

from oracle import fock
from workloads import hamiltonians as H

lcc = pytest.importorskip("paper_1509_00216_amd.lcc")
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    try:
        return lcc.library()
    except ImportError as e:
        pytest.skip(str(e))


def test_exports_every_declared_symbol():
    lib = _lib()
    header = open(os.path.join(ROOT, "include", "mpslcc.h")).read()
    declared = set(re.findall(r"\b(lcc_[a-z0-9_]+)\s*\(", header))
    assert declared, "no declarations found"
    for name in sorted(declared):
        assert hasattr(lib, name), name
    assert declared == set(lcc.EXPORTS)


def _dense_mpo(ham, K):
    partial = {0: np.ones((1, 1))}
    for j in range(K):
        wi, wo, m = ham.site_mpo(j)
        nxt = {}
        for a, b, mm in zip(wi, wo, m):
            if a in partial:
                nxt[b] = nxt.get(b, 0.0) + np.kron(partial[a], mm)
        partial = nxt
    assert list(partial) == [0]
    return partial[0]


@pytest.mark.parametrize("make,switch", [
    (lambda: H.hubbard_chain(4, t=1.0, U=3.0, n_elec=4), -1),
    (lambda: H.random_ab_initio(4, 4, seed=5), -1),
    (lambda: H.random_ab_initio(5, 4, two_sz=2, seed=2), 2),
    (lambda: H.random_ab_initio(5, 5, two_sz=1, seed=3), 4),
    (lambda: H.rotate_orbitals(H.hubbard_chain(4, U=2.0, n_elec=3, two_sz=1), H.random_orthogonal(4, 3)), -1),
    (lambda: H.three_band(2, 1, n_holes=3, two_sz=1), -1),
    (lambda: dict(H.hubbard_chain(3, U=1.5, n_elec=2), e_const=0.75), -1),
])
def test_product_mpo_equals_fock_hamiltonian(make, switch):
    _lib()
    spec = make()
    ham = lcc.create_hamiltonian(None, spec, switch_bond=switch)
    K = spec["n_orb"]
    D = _dense_mpo(ham, K)
    basis = fock.sector_basis(K, spec["n_elec"], spec["two_sz"])
    idx = np.zeros(basis.size, dtype=np.int64)
    for j in range(K):
        idx = idx * 4 + ((basis >> (2 * j)) & 1) + 2 * ((basis >> (2 * j + 1)) & 1)
    Hs = fock.hamiltonian_matrix(spec, basis).toarray()
    assert np.abs(D[np.ix_(idx, idx)] - Hs).max() < 1e-12 * max(1.0, np.abs(Hs).max())
    # charge bookkeeping: every entry maps channel shifts consistently with its local operator
    qn = [(0, 0), (1, 1), (1, -1), (2, 0)]
    for j in range(K):
        dn_l, dz_l = ham.channels(j)
        dn_r, dz_r = ham.channels(j + 1)
        wi, wo, m = ham.site_mpo(j)
        for a, b, mm in zip(wi, wo, m):
            for sp, s in zip(*np.nonzero(mm)):
                assert dn_r[b] - dn_l[a] == qn[sp][0] - qn[s][0]
                assert dz_r[b] - dz_l[a] == qn[sp][1] - qn[s][1]


def test_bond_dimensions():
    _lib()
    ham = lcc.create_hamiltonian(None, H.hubbard_chain(8, U=4.0, n_elec=8))
    assert list(ham.bond_dims()) == [1, 6, 6, 6, 6, 6, 6, 6, 1]
    ham = lcc.create_hamiltonian(None, H.random_ab_initio(24, 12, seed=1003))
    d = ham.bond_dims()
    assert d[0] == 1 and d[24] == 1
    # O(k^2): 2 + 4k one-operator channels + (2k)^2/2 two-operator channels at the centre
    assert 1100 <= d[12] <= 1300


def test_argument_errors():
    _lib()
    spec = H.hubbard_chain(4, U=1.0, n_elec=4)
    with pytest.raises(lcc.LccError) as e:
        lcc.create_hamiltonian(None, dict(spec, two_sz=1))
    assert e.value.code == -2
    with pytest.raises(lcc.LccError) as e:
        lcc.create_hamiltonian(None, dict(spec, h=np.full((4, 4), np.nan)))
    assert e.value.code == -4
    ctx = lcc.Context(device=-1)
    ham = ctx.create_hamiltonian(spec)
    from workloads import mps as M
    mps = M.random_mps(4, 4, 0, 8, seed=1)
    with pytest.raises(lcc.LccError) as e:
        ctx.build_environments(ham, mps)
    assert e.value.code == -7
    # planner and scheduling setters validate their arguments on a host-only context
    ctx.set_plan(8192.0, 1024, 1, 1)
    ctx.set_plan(8192.0, 1024, 1, 2)
    ctx.set_overlap(0)
    for bad in ((float("nan"), 1024, 0, 0), (-1.0, 1024, 0, 0), (2048.0, 0, 0, 0), (2048.0, 1024, 2, 0),
                (2048.0, 1024, 0, 3), (2048.0, 1024, 0, -1)):
        with pytest.raises(lcc.LccError) as e:
            ctx.set_plan(*bad)
        assert e.value.code == -1, bad
    for bad in (-1, 9):
        with pytest.raises(lcc.LccError) as e:
            ctx.set_overlap(bad)
        assert e.value.code == -1
