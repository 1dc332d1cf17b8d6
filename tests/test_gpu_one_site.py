"""The one-site local problem on the device (lcc_build_environments_one_site: the unknown is one
site tensor, Implementation section, local-derivative figure and sweep) against the oracle's
one-site effective Hamiltonian (oracle.fock.effective_hamiltonian_one_site, pinned in
test_oracle_one_site.py) and, at full size, its block-sparse route through the two-site
environments (oracle.blocksparse.one_site_apply).

* H1 x in FP64 / FP32 / BF16x3 at the first, a middle and the last site (bars 1e-12 / 1e-5 /
  1e-4 relative, as for the two-site product), and at the 4x4 Hubbard model with M = 500;
* the exact ground state: its site tensor is mapped to E0 times itself;
* the local solve (FP64 and mixed) against the dense solution of the same system, and the
  lowest eigenpair against dense diagonalisation.
"""
import numpy as np
import pytest

from gpu_common import need_gpu, rel, say, to_dev
from oracle import blocksparse as BS
from oracle import fock
from oracle import mpo as OM
from oracle import solve as OS
from workloads import configs as C
from workloads import hamiltonians as H
from workloads import mps as M

pytestmark = pytest.mark.gpu

SYSTEMS = {
    "abinitio_k6_m10": lambda: (H.random_ab_initio(6, 6, seed=21), M.random_mps(6, 6, 0, 10, seed=22, center=2)),
    "hubbard_4x2_m16": lambda: (H.hubbard_2d(4, 2, U=4.0, n_elec=7, two_sz=1),
                                M.random_mps(8, 7, 1, 16, seed=8, center=3)),
}


def _keys(m1):
    return [(a, s, 0, b) for a, s, b in M.one_site_blocks(m1)]


def _apply(torch, env, xf, prec):
    dt = torch.float64 if prec == "fp64" else torch.float32
    x = to_dev(torch, xf, dt)
    y = torch.empty_like(x)
    env.apply_heff(x, y, prec)
    return y.double().cpu().numpy()


@pytest.mark.parametrize("name", sorted(SYSTEMS))
@pytest.mark.parametrize("where", ["first", "middle", "last"])
def test_apply_vs_dense(name, where):
    torch, lcc = need_gpu()
    spec, mps = SYSTEMS[name]()
    K = spec["n_orb"]
    site = {"first": 0, "middle": mps["center"], "last": K - 1}[where]
    m1 = M.canonical_at(mps, site)
    keys = _keys(m1)
    H1 = fock.effective_hamiltonian_one_site(spec, m1, keys)
    ctx = lcc.Context(0)
    env = ctx.build_environments_one_site(ctx.create_hamiltonian(spec), m1, site)
    assert env.n == H1.shape[0]
    x = M.random_one_site_vector(m1, 3)
    xf = env.pack(x)
    yref = env.pack(BS.unflatten(H1 @ BS.flatten(x, keys), x, keys))
    err = {p: rel(_apply(torch, env, xf, p), yref) for p in ("fp64", "fp32", "bf16x3")}
    say(f"[one-site] {name} site {site} n={env.n}: {err}")
    assert err["fp64"] <= 1e-12
    assert err["fp32"] <= 1e-5
    assert err["bf16x3"] <= 1e-4


def test_apply_full_size_vs_blocksparse():
    torch, lcc = need_gpu()
    spec, mps = C.make("hubbard2d_4x4_m500")
    site = mps["center"]
    m1 = M.canonical_at(mps, site)
    ctx = lcc.Context(0)
    say("[one-site] hubbard2d 4x4 M=500: build")
    env = ctx.build_environments_one_site(ctx.create_hamiltonian(spec), m1, site)
    x = M.random_one_site_vector(m1, 4)
    say(f"[one-site] n={env.n}: oracle")
    yref = env.pack(BS.one_site_apply(spec, m1, OM.build_mpo(spec), x))
    xf = env.pack(x)
    err = {p: rel(_apply(torch, env, xf, p), yref) for p in ("fp64", "fp32", "bf16x3")}
    say(f"[one-site] full size errors {err}")
    assert err["fp64"] <= 1e-12
    assert err["fp32"] <= 1e-5
    assert err["bf16x3"] <= 1e-4


@pytest.mark.parametrize("site", [0, 3, 5])
def test_exact_ground_state_site_tensor(site):
    torch, lcc = need_gpu()
    spec = dict(H.random_ab_initio(6, 6, two_sz=0, seed=11), e_const=0.3)
    basis = fock.sector_basis(6, 6, 0)
    w, V = np.linalg.eigh(fock.hamiltonian_matrix(spec, basis).toarray())
    full = np.zeros(4 ** 6)
    full[fock.config_index(basis, 6)] = V[:, 0]
    m1 = M.canonical_at(M.mps_from_amplitudes(full, 6, 6, 0), site)
    ctx = lcc.Context(0)
    env = ctx.build_environments_one_site(ctx.create_hamiltonian(spec), m1, site)
    a = env.pack({(il, s, 0, ir): A for il, s, ir, A in m1["sites"][site]})
    y = _apply(torch, env, a, "fp64")
    say(f"[one-site] exact ground state, site {site}: |H1 a - E0 a| = {np.abs(y - w[0] * a).max():.2e}")
    assert np.abs(y - w[0] * a).max() <= 1e-11 * abs(w[0])


def test_solve_and_eigenpair_vs_dense():
    torch, lcc = need_gpu()
    spec, mps = SYSTEMS["hubbard_4x2_m16"]()
    site = mps["center"]
    m1 = M.canonical_at(mps, site)
    keys = _keys(m1)
    H1 = fock.effective_hamiltonian_one_site(spec, m1, keys)
    w = np.linalg.eigvalsh(H1)
    e0 = w[0] - 0.5
    bvec = M.random_one_site_vector(m1, 9)
    bflat = BS.flatten(bvec, keys)
    xstar = np.linalg.solve(H1 - e0 * np.eye(H1.shape[0]), bflat)
    jstar = -float(bflat @ xstar)
    ctx = lcc.Context(0)
    env = ctx.build_environments_one_site(ctx.create_hamiltonian(spec), m1, site)
    b = to_dev(torch, env.pack(bvec), torch.float64)
    for prec in ("fp64", "fp32"):
        x = torch.zeros_like(b)
        info = env.solve_local_lcc(b, e0, x, precision=prec, tol=1e-11, max_iter=2000, inner_tol=1e-4, max_outer=50)
        say(f"[one-site] solve {prec}: J {info['hylleraas']:.14f} (dense {jstar:.14f}), {info['iterations']} it")
        assert info["status"] == "LCC_OK"
        assert abs(info["hylleraas"] - jstar) <= 1e-10 * abs(jstar)
        assert rel(x.cpu().numpy(), env.pack(BS.unflatten(xstar, bvec, keys))) <= 1e-9
    x = torch.zeros_like(b)
    info = env.lowest_eigenpair(x, steps=40, max_restarts=40, tol=1e-11, seed=3)
    say(f"[one-site] eigenpair {info['theta']:.14f} (dense {w[0]:.14f})")
    assert info["status"] == "LCC_OK"
    assert abs(info["theta"] - w[0]) <= 1e-10


def test_tuner_and_batches_take_one_site_environments():
    """A one-site environment goes through every entry point that takes an environment: the
    autotuner (tuned plan = oracle), a batch with a two-site member and the one-shot batched solve
    (energies = the dense solution of each system)."""
    torch, lcc = need_gpu()
    spec, mps = SYSTEMS["hubbard_4x2_m16"]()
    site = mps["center"]
    m1 = M.canonical_at(mps, site)
    keys = _keys(m1)
    H1 = fock.effective_hamiltonian_one_site(spec, m1, keys)
    ctx = lcc.Context(0)
    ham = ctx.create_hamiltonian(spec)
    env = ctx.build_environments_one_site(ham, m1, site)
    info = env.autotune("fp32", reps=2)
    say(f"[one-site] autotune {info}")
    x = M.random_one_site_vector(m1, 6)
    yref = env.pack(BS.unflatten(H1 @ BS.flatten(x, keys), x, keys))
    assert rel(_apply(torch, env, env.pack(x), "fp64"), yref) <= 1e-12
    assert rel(_apply(torch, env, env.pack(x), "fp32"), yref) <= 1e-5
    # a batch of the one-site problem and the two-site problem of the same MPS
    blocks2 = M.two_site_blocks(mps)
    H2 = fock.effective_hamiltonian(spec, mps, blocks2)
    env2 = ctx.build_environments(ham, mps)
    probs = []
    for e, Hm, vec in ((env, H1, M.random_one_site_vector(m1, 7)), (env2, H2, M.random_two_site_vector(mps, 8))):
        k = keys if e is env else blocks2
        e0 = np.linalg.eigvalsh(Hm)[0] - 0.5
        bflat = BS.flatten(vec, k)
        jstar = -float(bflat @ np.linalg.solve(Hm - e0 * np.eye(Hm.shape[0]), bflat))
        probs.append((e, e0, to_dev(torch, e.pack(vec), torch.float64), jstar))
    for runner in ("batch", "one-shot"):
        xs = [torch.zeros_like(b) for _, _, b, _ in probs]
        args = ([b for _, _, b, _ in probs], [e0 for _, e0, _, _ in probs], xs)
        if runner == "batch":
            status, infos = lcc.Batch(ctx, [e for e, _, _, _ in probs]).solve(*args, precision="fp32", tol=1e-10,
                                                                               max_iter=2000)
        else:
            status, infos = lcc.solve_local_lcc_batched([e for e, _, _, _ in probs], *args, precision="fp32",
                                                        tol=1e-10, max_iter=2000)
        say(f"[one-site] {runner}: {[i['hylleraas'] for i in infos]} vs {[j for _, _, _, j in probs]}")
        assert status == "LCC_OK"
        for (_, _, _, jstar), inf in zip(probs, infos):
            assert abs(inf["hylleraas"] - jstar) <= 1e-8 * abs(jstar)


def _identity_spec(spec):
    n = spec["n_orb"]
    return {"name": "identity", "n_orb": n, "h": np.zeros((n, n)), "eri": None, "u": None, "e_const": 1.0,
            "n_elec": spec["n_elec"], "two_sz": spec["two_sz"]}


@pytest.mark.parametrize("site", [0, 2, 5])
def test_one_site_transition_rhs_vs_fock(site):
    """One-site transition environments (lcc_build_transition_environments_one_site): applied to
    the ket's own site tensor they give u = P1^T H Phi0 and, with H = 1, v = P1^T Phi0, where P1 is
    the bra's one-site isometry (the first-order right-hand side of the one-site problem); the
    ket has other bond dimensions and its own gauge.  Bars: 1e-12 relative (FP64), 1e-5 (FP32)."""
    torch, lcc = need_gpu()
    spec = H.random_ab_initio(6, 6, seed=21)
    bra = M.canonical_at(M.random_mps(6, 6, 0, 10, seed=22, center=2), site)
    ket = M.random_mps(6, 6, 0, 6, seed=23, center=1)
    keys = _keys(bra)
    u_ref, v_ref, _ = fock.first_order_vectors(spec, bra, ket, keys, one_site=True)
    ctx = lcc.Context(0)
    tenv = lcc.build_transition_environments_one_site(ctx, ctx.create_hamiltonian(spec), bra, ket, site)
    ienv = lcc.build_transition_environments_one_site(ctx, ctx.create_hamiltonian(_identity_spec(spec)), bra, ket,
                                                      site)
    assert tenv.transition
    x0 = torch.zeros(tenv.n_in, dtype=torch.float64, device="cuda:0")
    tenv.ket_tensor(x0)
    u = torch.empty(tenv.n, dtype=torch.float64, device="cuda:0")
    v = torch.empty(tenv.n, dtype=torch.float64, device="cuda:0")
    tenv.apply_heff(x0, u, "fp64")
    ienv.apply_heff(x0, v, "fp64")
    u32 = torch.empty(tenv.n, dtype=torch.float32, device="cuda:0")
    tenv.apply_heff(x0.float(), u32, "fp32")
    torch.cuda.synchronize()
    tmpl = {k: np.zeros((bra["bonds"][site][k[0]][2], bra["bonds"][site + 1][k[3]][2])) for k in keys}
    pk = lambda flat: tenv.pack(BS.unflatten(flat, tmpl, keys))
    eu, ev = rel(u.cpu().numpy(), pk(u_ref)), rel(v.cpu().numpy(), pk(v_ref))
    say(f"[one-site] transition at site {site}: u rel {eu:.2e}, v rel {ev:.2e}, |v| {np.linalg.norm(v_ref):.4f}")
    assert eu <= 1e-12 and ev <= 1e-12
    assert rel(u32.double().cpu().numpy(), pk(u_ref)) <= 1e-5


def test_one_site_first_order_local_solve():
    """The first-order local problem of one site tensor end to end: b = -(u - e1 v) and v from the
    one-site transition environments, then Q(H1 - E0)Q x = Q b with Q = 1 - v v^T / |v|^2 on the
    one-site environment, in FP64 and mixed precision, against the dense solution of the same
    equation built from the oracle's u, v, e1 and one-site H_eff (J within 1e-9, x orthogonal to v)."""
    torch, lcc = need_gpu()
    spec = H.random_ab_initio(6, 6, seed=21)
    site = 2
    bra = M.canonical_at(M.random_mps(6, 6, 0, 10, seed=22, center=2), site)
    ket = M.random_mps(6, 6, 0, 6, seed=23, center=1)
    keys = _keys(bra)
    u_ref, v_ref, e1 = fock.first_order_vectors(spec, bra, ket, keys, one_site=True)
    H1 = fock.effective_hamiltonian_one_site(spec, bra, keys)
    e0 = float(np.linalg.eigvalsh(H1)[0]) - 0.5
    bref = -(u_ref - e1 * v_ref)
    vh = v_ref / np.linalg.norm(v_ref)
    xs = OS.dense_solution(H1, bref, e0, vh)
    jstar = OS.hylleraas(OS.make_operator(lambda z: H1 @ z, e0, vh), xs, OS.project(vh, bref))
    ctx = lcc.Context(0)
    ham = ctx.create_hamiltonian(spec)
    tenv = lcc.build_transition_environments_one_site(ctx, ham, bra, ket, site)
    ienv = lcc.build_transition_environments_one_site(ctx, ctx.create_hamiltonian(_identity_spec(spec)), bra, ket,
                                                      site)
    x0 = torch.zeros(tenv.n_in, dtype=torch.float64, device="cuda:0")
    tenv.ket_tensor(x0)
    u = torch.empty(tenv.n, dtype=torch.float64, device="cuda:0")
    v = torch.empty(tenv.n, dtype=torch.float64, device="cuda:0")
    tenv.apply_heff(x0, u, "fp64")
    ienv.apply_heff(x0, v, "fp64")
    b = -(u - e1 * v)
    vhat = v / v.norm()
    env = ctx.build_environments_one_site(ham, bra, site)
    for prec in ("fp64", "fp32"):
        x = torch.zeros_like(b)
        info = env.solve_local_lcc(b, e0, x, v=vhat, precision=prec, tol=1e-12, max_iter=2000, inner_tol=1e-4,
                                   max_outer=100)
        say(f"[one-site] first-order solve {prec}: J {info['hylleraas']:.15f} dense {jstar:.15f}")
        assert info["status"] == "LCC_OK"
        assert abs(info["hylleraas"] - jstar) <= 1e-9
        assert abs(float(vhat @ x)) <= 1e-10 * float(x.norm())
