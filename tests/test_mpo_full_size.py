"""MPOs at the full ab initio size (K = 24, the benchmarked Hamiltonian) pinned by the
Slater-Condon rules: <D'|H|D> between occupation-number states, read off the MPO by contracting
its site tensors with the two states' local indices, must equal the textbook matrix elements
built from h and (ij|kl) directly.  The rules themselves are first checked against the oracle's
Fock-space Hamiltonian (O1) on every pair of states of small systems.

This covers the oracle's two-sided MPO (oracle.mpo.build_mpo_twosided, the MPO of the
full-size oracle contraction) and the library's MPO (read through the C ABI on a host-only
context), at the size where the dense contraction of the small-system pins is out of reach.
"""
import numpy as np
import pytest

from oracle import fock
from oracle import mpo as OM
from slater_condon import SlaterCondon, local_index, sample_pairs
from workloads import configs as C
from workloads import hamiltonians as H


def _site_arrays(mpo):
    K = mpo["n_sites"]
    out = []
    for j in range(K):
        keys = list(mpo["W"][j])
        win = np.array([k[0] for k in keys], dtype=np.int64)
        wout = np.array([k[1] for k in keys], dtype=np.int64)
        mats = np.array([np.asarray(mpo["W"][j][k]).reshape(16) for k in keys])
        out.append((win, wout, mats, len(mpo["dq"][j + 1])))
    return out


def mpo_element(arrays, bra, ket):
    v = np.ones(1)
    for j, (win, wout, mats, dout) in enumerate(arrays):
        col = 4 * local_index(bra, j) + local_index(ket, j)
        v = np.bincount(wout, weights=mats[:, col] * v[win], minlength=dout)
    return float(v[0])


@pytest.mark.parametrize("make", [
    lambda: H.random_ab_initio(5, 4, two_sz=0, seed=7),
    lambda: H.random_ab_initio(6, 5, two_sz=1, seed=8),
    lambda: dict(H.three_band(2, 1, n_holes=3, two_sz=1), e_const=0.3),
])
def test_slater_condon_rules_match_fock_space(make):
    spec = make()
    basis = fock.sector_basis(spec["n_orb"], spec["n_elec"], spec["two_sz"])
    Hs = fock.hamiltonian_matrix(spec, basis).toarray()
    sc = SlaterCondon(spec)
    ref = np.array([[sc.element(int(b), int(k)) for k in basis] for b in basis])
    assert np.abs(ref - Hs).max() <= 1e-12 * max(1.0, np.abs(Hs).max())


@pytest.fixture(scope="module")
def headline():
    spec, _ = C.make("abinitio_k24_m1000")
    pairs = sample_pairs(spec["n_orb"], spec["n_elec"], spec["two_sz"], 30, seed=2024)
    sc = SlaterCondon(spec)
    ref = np.array([sc.element(b, k) for b, k in pairs])
    assert np.count_nonzero(ref) > len(pairs) // 2
    return spec, pairs, ref


def test_oracle_twosided_mpo_full_size(headline):
    spec, pairs, ref = headline
    mpo = OM.build_mpo_twosided(spec)
    assert max(len(c) for c in mpo["channels"]) <= 2 * spec["n_orb"] ** 2 + 4 * spec["n_orb"] + 2
    arr = _site_arrays(mpo)
    got = np.array([mpo_element(arr, b, k) for b, k in pairs])
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def test_library_mpo_full_size(headline):
    lcc = pytest.importorskip("paper_1509_00216_amd.lcc")
    try:
        lcc.library()
    except ImportError as e:
        pytest.skip(str(e))
    spec, pairs, ref = headline
    ham = lcc.create_hamiltonian(lcc.Context(-1), spec)
    K = spec["n_orb"]
    dims = ham.bond_dims()
    mpo = {"n_sites": K, "dq": [[0] * int(d) for d in dims], "W": []}
    for j in range(K):
        wi, wo, m = ham.site_mpo(j)
        mpo["W"].append({(int(a), int(b)): mm for a, b, mm in zip(wi, wo, m)})
    arr = _site_arrays(mpo)
    got = np.array([mpo_element(arr, b, k) for b, k in pairs])
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
