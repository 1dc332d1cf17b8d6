"""Pins of the oracle's exact flop counts (oracle.flops).

The counts are integers computed from block tables only.  They are pinned to
* the multiply-add work that the oracle's two contractions of H_eff x actually perform
  (the canonical L, W, R order and the factorisation over the middle MPO bond, with either
  enlarged operator applied first), counted
  product by product while they run, on systems where both contractions are also checked
  against the Fock-space H_eff of O1 (so the counted work is a correct contraction);
* the O(M^3) cost of the H0 term (Implementation section): scaling every sector dimension
  by 2 multiplies each GEMM count by exactly 8 and the W-mixing count by exactly 4.
"""
import numpy as np
import pytest

from oracle import blocksparse as BS
from oracle import flops as OF
from oracle import fock
from oracle import mpo as OM
from workloads import configs as C
from workloads import hamiltonians as H
from workloads import mps as M

CASES = {
    "chain8_complete": lambda: C.make("hubbard1d_k8_m64"),
    "abinitio_k6_m12": lambda: (H.random_ab_initio(6, 6, seed=21), M.random_mps(6, 6, 0, 12, seed=22)),
    "threeband_2x1_m10": lambda: (H.three_band(2, 1, n_holes=3, two_sz=1), M.random_mps(6, 3, 1, 10, seed=4)),
    "hubbard_4x2_m16_offcentre": lambda: (H.hubbard_2d(4, 2, U=4.0, n_elec=7, two_sz=1),
                                          M.random_mps(8, 7, 1, 16, seed=8, center=2)),
}


def _o1(spec, mps, x):
    blocks = M.two_site_blocks(mps)
    heff = fock.effective_hamiltonian(spec, mps, blocks)
    return heff @ BS.flatten(x, blocks), blocks


@pytest.mark.parametrize("name", sorted(CASES))
def test_counts_equal_the_work_of_both_contractions(name):
    spec, mps = CASES[name]()
    mpo = OM.build_mpo(spec)
    x = M.random_two_site_vector(mps, 5)
    y1, blocks = _o1(spec, mps, x)
    # canonical order
    cnt = {}
    y = BS.Environments(spec, mps, mpo).apply(x, counter=cnt)
    assert np.linalg.norm(BS.flatten(y, blocks) - y1) <= 1e-13 * np.linalg.norm(y1)
    can = OF.canonical_flops(mps, mpo)
    assert (can["k1"], can["k2"], can["k3"]) == (cnt["k1"], cnt["k2"], cnt["k3"])
    assert min(can["k1"], can["k2"], can["k3"]) > 0
    # middle-bond factorisation, both orders
    for order in ("left", "right"):
        cnt2 = {}
        y2 = BS.MiddleBondEnvironments(spec, mps, mpo).apply(x, counter=cnt2, order=order)
        assert np.linalg.norm(BS.flatten(y2, blocks) - y1) <= 1e-13 * np.linalg.norm(y1)
        fac = OF.factorised_flops(mps, mpo, order)
        assert (fac["left"], fac["right"]) == (cnt2["left"], cnt2["right"])
        assert fac["left"] > 0 and fac["right"] > 0


def test_counts_scale_as_the_cube_of_the_bond_dimension():
    spec, mps = C.make("hubbard2d_4x4_m500", m_max=30)
    mpo = OM.build_mpo(spec)
    doubled = dict(mps, bonds=[[(n, z, 2 * d) for n, z, d in bond] for bond in mps["bonds"]])
    a, b = OF.canonical_flops(mps, mpo), OF.canonical_flops(doubled, mpo)
    assert (b["k1"], b["k2"], b["k3"]) == (8 * a["k1"], 4 * a["k2"], 8 * a["k3"])
    for order in ("left", "right"):
        fa, fb = OF.factorised_flops(mps, mpo, order), OF.factorised_flops(doubled, mpo, order)
        assert (fb["left"], fb["right"]) == (8 * fa["left"], 8 * fa["right"])


def test_count_is_independent_of_vector_values():
    # the count is a property of the block tables: a planted zero block of L still counts,
    # as the contraction forms the product regardless of the entries
    spec, mps = CASES["abinitio_k6_m12"]()
    mpo = OM.build_mpo(spec)
    x = M.random_two_site_vector(mps, 9)
    for k in list(x)[::3]:
        x[k] = np.zeros_like(x[k])
    for order in ("left", "right"):
        cnt = {}
        BS.MiddleBondEnvironments(spec, mps, mpo).apply(x, counter=cnt, order=order)
        fac = OF.factorised_flops(mps, mpo, order)
        assert (fac["left"], fac["right"]) == (cnt["left"], cnt["right"])


@pytest.mark.parametrize("name", ["abinitio_k6_m12", "hubbard_4x2_m16_offcentre", "chain8_complete"])
def test_one_site_counts_equal_the_work_of_the_contraction(name):
    # the one-site problem (right enlarged operator = R): the factorised contraction equals the
    # dense one-site H_eff of O1, and its counted work equals the integer count, in both orders
    spec, mps = CASES[name]()
    m1 = M.canonical_at(mps, mps["center"])
    mpo = OM.build_mpo(spec)
    keys = [(a, s, 0, b) for a, s, b in M.one_site_blocks(m1)]
    yd = fock.effective_hamiltonian_one_site(spec, m1, keys) @ BS.flatten(M.random_one_site_vector(m1, 5), keys)
    x = M.random_one_site_vector(m1, 5)
    for order in ("left", "right"):
        cnt = {}
        y = BS.MiddleBondEnvironments(spec, m1, mpo, one_site=True).apply(x, counter=cnt, order=order)
        assert np.linalg.norm(BS.flatten(y, keys) - yd) <= 1e-13 * np.linalg.norm(yd)
        fac = OF.factorised_flops(m1, mpo, order, one_site=True)
        assert (fac["left"], fac["right"]) == (cnt["left"], cnt["right"])
        assert fac["left"] > 0 and fac["right"] > 0
