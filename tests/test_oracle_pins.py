"""Pins of the CPU oracle against facts fixed outside it (closed forms, symmetries, ED).

These run without a GPU.  Each test names the mathematical fact it relies on; a plausible
mistake in the oracle (a sign, an index order, a dropped factor, a transposed operand)
breaks at least one of them (see test_planted_mistakes).
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import blocksparse as BS
from oracle import fock
from oracle import mpo as OM
from oracle import solve as OS
from workloads import configs as C
from workloads import hamiltonians as H
from workloads import mps as M

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")))


def sector_to_config(basis, K):
    idx = np.zeros(basis.size, dtype=np.int64)
    for j in range(K):
        s = ((basis >> (2 * j)) & 1) + 2 * ((basis >> (2 * j + 1)) & 1)
        idx = idx * 4 + s
    return idx


def test_hubbard_dimer_closed_form():
    e = fock.ground_energy(H.hubbard_chain(2, t=1.0, U=4.0, n_elec=2))[0]
    assert abs(e - GOLD["hubbard_dimer_t1_U4_ground"]) < 1e-12


def test_tight_binding_closed_form():
    e = fock.ground_energy(H.hubbard_chain(8, t=1.0, U=0.0, n_elec=8))[0]
    assert abs(e - GOLD["tight_binding_obc_L8_halffilling_ground"]) < 1e-11


def test_particle_hole_symmetry_and_trace():
    spec = H.hubbard_chain(8, t=1.0, U=4.0, n_elec=8)
    Hm = fock.hamiltonian_matrix(spec).toarray()
    assert Hm.shape[0] == GOLD["hubbard_chain_L8_sector_dim"]
    w = np.linalg.eigvalsh(Hm)
    assert abs(w[0] + w[-1] - GOLD["hubbard_chain_L8_U4_lmin_plus_lmax"]) < 1e-10
    assert abs(np.trace(Hm) - GOLD["hubbard_chain_L8_U4_trace"]) < 1e-8


def test_constant_two_body_is_pair_count():
    # (ij|kl) = V d_ij d_kl  =>  1/2 V sum a+_i a+_k a_k a_i = V N (N - 1) / 2 on every state
    K, N, V = 4, 3, 0.7
    eri = np.zeros((K, K, K, K))
    for i in range(K):
        for k in range(K):
            eri[i, i, k, k] = V
    spec = H._spec("pairs", np.zeros((K, K)), N, 1, eri=eri)
    Hm = fock.hamiltonian_matrix(spec).toarray()
    assert np.allclose(Hm, np.eye(Hm.shape[0]) * V * N * (N - 1) / 2, atol=1e-13)


def test_orbital_rotation_invariance_pins_two_body_convention():
    # the on-site U written as (ii|ii) and rotated to a dense (ij|kl) must keep the spectrum
    base = H.hubbard_chain(4, t=1.0, U=3.0, n_elec=4)
    rot = H.rotate_orbitals(base, H.random_orthogonal(4, 11))
    w0 = np.linalg.eigvalsh(fock.hamiltonian_matrix(base).toarray())
    w1 = np.linalg.eigvalsh(fock.hamiltonian_matrix(rot).toarray())
    assert np.abs(w0 - w1).max() < 1e-11


@pytest.mark.parametrize("make", [
    lambda: H.hubbard_chain(4, t=1.0, U=3.0, n_elec=4),
    lambda: H.random_ab_initio(4, 4, seed=5),
    lambda: H.rotate_orbitals(H.hubbard_chain(4, U=2.0, n_elec=3, two_sz=1), H.random_orthogonal(4, 3)),
    lambda: H.three_band(2, 1, n_holes=3, two_sz=1),
])
@pytest.mark.parametrize("builder", ["prefix", "twosided", "twosided_switch1", "twosided_switch3"])
def test_oracle_mpo_contracts_to_fock_hamiltonian(make, builder):
    spec = make()
    if builder == "prefix":
        mpo = OM.build_mpo(spec)
    else:
        mpo = OM.build_mpo_twosided(spec, {"twosided": None, "twosided_switch1": 1, "twosided_switch3": 3}[builder])
    D = OM.dense_operator(mpo)
    basis = fock.sector_basis(spec["n_orb"], spec["n_elec"], spec["two_sz"])
    ci = sector_to_config(basis, spec["n_orb"])
    Hs = fock.hamiltonian_matrix(spec, basis).toarray()
    assert np.abs(D[np.ix_(ci, ci)] - Hs).max() < 1e-12 * max(1.0, np.abs(Hs).max())
    # the MPO conserves N and Sz: no amplitude leaves the sector
    other = np.setdiff1d(np.arange(D.shape[0]), ci)
    assert np.abs(D[np.ix_(other, ci)]).max() < 1e-14
    # channel shifts agree with the entries: <s'|W^{w,w'}|s> != 0 only if dq(w') = dq(w) + qn(s') - qn(s)
    for j, Wj in enumerate(mpo["W"]):
        for (a, b), m in Wj.items():
            for sp in range(4):
                for s in range(4):
                    if m[sp, s] != 0.0:
                        assert mpo["dq"][j + 1][b][0] == mpo["dq"][j][a][0] + OM.LOCAL_QN[sp][0] - OM.LOCAL_QN[s][0]
                        assert mpo["dq"][j + 1][b][1] == mpo["dq"][j][a][1] + OM.LOCAL_QN[sp][1] - OM.LOCAL_QN[s][1]


def test_generator_canonical_and_isometry():
    spec, mps = C.make("hubbard1d_k8_m64")
    assert BS.check_left_canonical(mps) < 1e-13
    assert BS.check_right_canonical(mps) < 1e-13
    blocks = M.two_site_blocks(mps)
    basis = fock.sector_basis(8, 8, 0)
    P = fock.two_site_isometry(mps, basis, blocks)
    assert P.shape == (4900, 4900)
    assert np.abs(P.T @ P - np.eye(P.shape[1])).max() < 1e-12


@pytest.fixture(scope="module")
def chain8():
    spec, mps = C.make("hubbard1d_k8_m64")
    blocks = M.two_site_blocks(mps)
    heff = fock.effective_hamiltonian(spec, mps, blocks)
    return spec, mps, blocks, heff


def test_complete_basis_heff_spectrum_is_ed(chain8):
    spec, mps, blocks, heff = chain8
    w = np.linalg.eigvalsh(heff)
    ed = np.linalg.eigvalsh(fock.hamiltonian_matrix(spec).toarray())
    assert np.abs(w - ed).max() < 1e-10
    assert abs(w[0] + w[-1] - GOLD["hubbard_chain_L8_U4_lmin_plus_lmax"]) < 1e-10
    assert abs(np.trace(heff) - GOLD["hubbard_chain_L8_U4_trace"]) < 1e-7


def test_blocksparse_matches_fock(chain8):
    spec, mps, blocks, heff = chain8
    env = BS.Environments(spec, mps, OM.build_mpo(spec))
    x = M.random_two_site_vector(mps, 7)
    y = BS.flatten(env.apply(x), blocks)
    y1 = heff @ BS.flatten(x, blocks)
    assert np.linalg.norm(y - y1) / np.linalg.norm(y1) < 1e-14


def test_blocksparse_matches_fock_ab_initio_truncated():
    spec = H.random_ab_initio(6, 6, seed=21)
    mps = M.random_mps(6, 6, 0, 12, seed=22)  # truncated bonds: P is a proper isometry
    blocks = M.two_site_blocks(mps)
    heff = fock.effective_hamiltonian(spec, mps, blocks)
    env = BS.Environments(spec, mps, OM.build_mpo(spec))
    x = M.random_two_site_vector(mps, 23)
    y = BS.flatten(env.apply(x), blocks)
    y1 = heff @ BS.flatten(x, blocks)
    assert np.linalg.norm(y - y1) / np.linalg.norm(y1) < 1e-13
    assert np.abs(heff - heff.T).max() < 1e-12 * np.abs(heff).max()


def test_number_operator_environments():
    # H = N-hat: H_eff x = N x exactly (isometry + particle-number conservation)
    spec = H.number_operator(10, 7, 1)
    mps = M.random_mps(10, 7, 1, 40, seed=5)
    env = BS.Environments(spec, mps, OM.build_mpo(spec))
    x = M.random_two_site_vector(mps, 6)
    y = env.apply(x)
    err = max(np.abs(y[k] - 7 * x[k]).max() for k in x)
    assert err < 1e-12


def test_interlacing_lower_bound_4x4():
    spec = H.hubbard_2d(4, 4, U=4.0, n_elec=14)
    mps = M.random_mps(16, 14, 0, 40, seed=9)
    env = BS.Environments(spec, mps, OM.build_mpo(spec))
    blocks = M.two_site_blocks(mps)
    tmpl = BS.two_site_template(mps, blocks)
    n = sum(v.size for v in tmpl.values())
    ap = lambda z: BS.flatten(env.apply(BS.unflatten(z, tmpl, blocks)), blocks)
    th, res, _ = OS.lanczos_lowest(ap, n, steps=80, seed=1)
    e_free = C.free_fermion_energy(spec["h"], 7, 7)
    assert abs(e_free - (-24.0)) < 1e-10  # U = 0 ground energy of the 4x4 torus, N = 14
    assert th - res >= e_free - 1e-9


def test_local_solve_spectral_formula(chain8):
    # complete basis, E0 = E_ED, Q projects out the ground state: x* = sum_k>0 (u_k.b)/(l_k - l_0) u_k
    spec, mps, blocks, heff = chain8
    w, U = np.linalg.eigh(heff)
    v = U[:, 0]
    rng = np.random.Generator(np.random.PCG64(3))
    b = rng.standard_normal(heff.shape[0])
    b /= np.linalg.norm(b)
    xs = OS.dense_solution(heff, b, w[0], v)
    ref = U[:, 1:] @ ((U[:, 1:].T @ b) / (w[1:] - w[0]))
    assert np.linalg.norm(xs - ref) / np.linalg.norm(ref) < 1e-10
    A = OS.make_operator(lambda z: heff @ z, w[0], v)
    x, it, rel, hist = OS.cg(A, b, tol=1e-12, v=v)
    assert rel <= 1e-12
    assert np.linalg.norm(x - ref) / np.linalg.norm(ref) < 1e-9
    assert all(hist[i + 1] <= hist[i] + 1e-12 for i in range(len(hist) - 1))
    jstar = OS.hylleraas(A, ref, OS.project(v, b))
    assert abs(jstar - (-(OS.project(v, b) @ ref))) < 1e-10
    # J(x) - J* = |x - x*|_A^2 >= 0 for any x
    z = ref + 0.01 * OS.project(v, rng.standard_normal(ref.size))
    d = z - ref
    assert OS.hylleraas(A, z, OS.project(v, b)) - jstar == pytest.approx(d @ A(d), rel=1e-8, abs=1e-12)


def test_cg_detects_indefinite():
    heff = np.diag([-1.0, 1.0, 2.0])
    A = OS.make_operator(lambda z: heff @ z, 0.0)
    with pytest.raises(ArithmeticError):
        OS.cg(A, np.array([1.0, 0.0, 0.0]))


def test_lanczos_lowest_is_the_lowest_eigenvalue(chain8):
    # two-sided: the Ritz value equals lambda_min of the dense matrix (not merely >= it), and
    # the reported residual is the true ||H u - theta u|| of the returned unit vector
    spec, mps, blocks, heff = chain8
    w = np.linalg.eigvalsh(heff)
    th, res, u = OS.lanczos_lowest(lambda z: heff @ z, heff.shape[0], steps=100, seed=2)
    assert abs(th - w[0]) <= 1e-10
    assert abs(np.linalg.norm(u) - 1.0) <= 1e-12
    assert abs(np.linalg.norm(heff @ u - th * u) - res) <= 1e-12
    assert res <= 1e-8
