"""GPU local LCC solve (conjugate gradients, FP64 and mixed precision with FP64 refinement)
against the oracle's exact solution, plus the error paths forced from the host.

Bars: energy |J(x_gpu) - J(x*)| <= 1e-8 for every precision after refinement;
FP64 solution relative error <= kappa * tol.
"""
import numpy as np
import pytest

from gpu_common import need_gpu, rel, say, to_dev
from oracle import blocksparse as BS
from oracle import fock
from oracle import mpo as OM
from oracle import solve as OS
from workloads import configs as C
from workloads import mps as M

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    torch, lcc = need_gpu()
    return lcc.Context(0)


@pytest.fixture(scope="module")
def chain(ctx):
    """Complete-basis chain: E0 = E_ED, Q removes the ED ground state (singular but consistent)."""
    spec, mps = C.make("hubbard1d_k8_m64")
    blocks = M.two_site_blocks(mps)
    heff = fock.effective_hamiltonian(spec, mps, blocks)
    w, U = np.linalg.eigh(heff)
    rng = np.random.Generator(np.random.PCG64(1001 + 3))
    b = rng.standard_normal(heff.shape[0])
    b /= np.linalg.norm(b)
    v = U[:, 0]
    xs = OS.dense_solution(heff, b, w[0], v)
    A = OS.make_operator(lambda z: heff @ z, w[0], v)
    jstar = OS.hylleraas(A, xs, OS.project(v, b))
    kappa = w[-1] / w[1] if w[1] > 0 else np.inf
    env = ctx.build_environments(ctx.create_hamiltonian(spec), mps)
    tmpl = BS.two_site_template(mps, blocks)
    to_layout = lambda flat: env.pack(BS.unflatten(flat, tmpl, blocks))
    return dict(spec=spec, mps=mps, env=env, b=to_layout(b), v=to_layout(v), e0=w[0], xs=to_layout(xs),
                jstar=jstar, kappa=(w[-1] - w[0]) / (w[1] - w[0]))


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3"])
def test_chain_solve_with_projector(chain, precision):
    torch, lcc = need_gpu()
    env = chain["env"]
    say(f"[solve] chain8 {precision}")
    b = to_dev(torch, chain["b"], torch.float64)
    v = to_dev(torch, chain["v"], torch.float64)
    x = torch.zeros_like(b)
    info = env.solve_local_lcc(b, chain["e0"], x, v=v, precision=precision, tol=1e-10)
    say(f"  {info}")
    assert info["status"] == "LCC_OK"
    assert info["rel_residual"] <= 1e-10
    xg = x.cpu().numpy()
    assert abs(info["hylleraas"] - chain["jstar"]) <= 1e-8
    assert abs(info["e2"] - chain["jstar"]) <= 1e-8
    assert rel(xg, chain["xs"]) <= max(1e-12, chain["kappa"] * 1e-10)
    if precision != "fp64":
        assert info["applies_low"] > 0 and info["outer"] >= 1


@pytest.mark.parametrize("name,m", [("hubbard2d_4x4_m500", 80), ("threeband_4x2_m2000", 200)])
def test_lattice_solve_vs_oracle_cg(ctx, name, m):
    torch, lcc = need_gpu()
    spec, mps = C.make(name, m_max=m)
    e0 = C.lower_bound_shift(spec, 0.5)
    say(f"[solve] {name}@M={m} e0={e0}")
    oenv = BS.Environments(spec, mps, OM.build_mpo(spec))
    blocks = M.two_site_blocks(mps)
    tmpl = BS.two_site_template(mps, blocks)
    apply_o = lambda z: BS.flatten(oenv.apply(BS.unflatten(z, tmpl, blocks)), blocks)
    bvec = M.random_two_site_vector(mps, 1002 + 7)
    bflat = BS.flatten(bvec, blocks)
    A = OS.make_operator(apply_o, e0)
    xo, it, relres, _ = OS.cg(A, bflat, tol=1e-13, max_iter=3000)
    jstar = OS.hylleraas(A, xo, bflat)
    env = ctx.build_environments(ctx.create_hamiltonian(spec), mps)
    bd = to_dev(torch, env.pack(bvec), torch.float64)
    xref = env.pack(BS.unflatten(xo, tmpl, blocks))
    for prec in ("fp64", "fp32", "bf16x3"):
        x = torch.zeros_like(bd)
        info = env.solve_local_lcc(bd, e0, x, precision=prec, tol=1e-10, max_iter=4000)
        say(f"  {prec}: {info}")
        assert info["status"] == "LCC_OK"
        assert abs(info["hylleraas"] - jstar) <= 1e-8
        assert rel(x.cpu().numpy(), xref) <= 1e-6


def test_indefinite_shift_is_reported(chain):
    torch, lcc = need_gpu()
    env = chain["env"]
    b = to_dev(torch, chain["b"], torch.float64)
    x = torch.zeros_like(b)
    with pytest.raises(lcc.LccError) as e:
        env.solve_local_lcc(b, 1e3, x, precision="fp64")  # e0 far above the spectrum
    assert e.value.code == -3


def test_nan_input_is_reported(chain):
    torch, lcc = need_gpu()
    env = chain["env"]
    bh = chain["b"].copy()
    bh[17] = np.nan
    b = to_dev(torch, bh, torch.float64)
    x = torch.zeros_like(b)
    with pytest.raises(lcc.LccError) as e:
        env.solve_local_lcc(b, chain["e0"], x)
    assert e.value.code == -4


def test_mixed_solve_graph_replays(chain):
    """The low-precision CG iteration is replayed from a graph kept with the environment: a second
    identical solve (replays of the first solve's graph, with the refreshes' eager work and
    synchronisations between them) repeats the first bit for bit; a different shift, another
    projector and the other low precision each need a new capture, and each such solve matches
    the plain FP64 solve of its own system (which runs no graph)."""
    torch, lcc = need_gpu()
    env = chain["env"]
    b = to_dev(torch, chain["b"], torch.float64)
    v = to_dev(torch, chain["v"], torch.float64)
    runs = []
    for _ in range(2):
        x = torch.zeros_like(b)
        info = env.solve_local_lcc(b, chain["e0"], x, v=v, precision="fp32", tol=1e-10, inner_tol=1e-2)
        runs.append((x.cpu().numpy(), info))
    assert runs[0][1]["status"] == "LCC_OK" and runs[0][1]["iterations"] > 4
    assert np.array_equal(runs[0][0], runs[1][0])
    assert runs[0][1]["hylleraas"] == runs[1][1]["hylleraas"]
    assert abs(runs[0][1]["hylleraas"] - chain["jstar"]) <= 1e-8
    for e0, vv, prec in ((chain["e0"] - 0.3, v, "fp32"), (chain["e0"] - 0.3, None, "fp32"),
                         (chain["e0"] - 0.3, None, "bf16x3"), (chain["e0"] - 0.7, None, "fp32")):
        x = torch.zeros_like(b)
        info = env.solve_local_lcc(b, e0, x, v=vv, precision=prec, tol=1e-10, inner_tol=1e-2)
        x64 = torch.zeros_like(b)
        ref = env.solve_local_lcc(b, e0, x64, v=vv, precision="fp64", tol=1e-10)
        say(f"[solve] graph replay e0 {e0:.4f} v={vv is not None} {prec}: J {info['hylleraas']:.14f} "
            f"fp64 {ref['hylleraas']:.14f}, {info['iterations']} it")
        assert info["status"] == "LCC_OK"
        assert abs(info["hylleraas"] - ref["hylleraas"]) <= 1e-10 * abs(ref["hylleraas"])


def test_max_iter_returns_not_converged(chain):
    torch, lcc = need_gpu()
    env = chain["env"]
    b = to_dev(torch, chain["b"], torch.float64)
    v = to_dev(torch, chain["v"], torch.float64)
    x = torch.zeros_like(b)
    info = env.solve_local_lcc(b, chain["e0"], x, v=v, max_iter=1)
    assert info["status"] == "LCC_NOT_CONVERGED"
    assert info["iterations"] == 1
    assert np.isfinite(x.cpu().numpy()).all() and float(x.abs().sum()) > 0


def test_bad_descriptors(ctx):
    torch, lcc = need_gpu()
    spec, mps = C.make("hubbard1d_k8_m64")
    ham = ctx.create_hamiltonian(spec)
    # a block whose right sector violates N/Sz conservation
    bad = dict(mps, sites=[list(s) for s in mps["sites"]])
    il, s, ir, a = bad["sites"][1][0]
    wrong = (ir + 1) % len(mps["bonds"][2])
    bad["sites"][1][0] = (il, s, wrong, np.zeros((mps["bonds"][1][il][2], mps["bonds"][2][wrong][2])))
    with pytest.raises(lcc.LccError) as e:
        ctx.build_environments(ham, bad)
    assert e.value.code in (-2, -1)
    # a left site that is not left-canonical
    scaled = dict(mps, sites=[list(s) for s in mps["sites"]])
    scaled["sites"][1] = [(a, b, c, 1.1 * d) for a, b, c, d in scaled["sites"][1]]
    with pytest.raises(lcc.LccError) as e:
        ctx.build_environments(ham, scaled)
    assert e.value.code == -1


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_zero_rhs_gives_zero_solution(chain, precision):
    """Degenerate right-hand side: Q b = 0 has the solution x = 0 and J = 0, with no iteration."""
    torch, lcc = need_gpu()
    env = chain["env"]
    b = torch.zeros(env.n, dtype=torch.float64, device="cuda:0")
    x = torch.full_like(b, 0.5)  # a non-zero guess is discarded
    info = env.solve_local_lcc(b, chain["e0"] - 1.0, x, precision=precision, tol=1e-10)
    assert info["status"] == "LCC_OK"
    assert info["iterations"] == 0
    assert info["hylleraas"] == 0.0 and info["e2"] == 0.0
    assert float(x.abs().max()) == 0.0


def test_batch_with_zero_rhs_member(chain, ctx):
    """A batch whose second member has b = 0: that member stays at x = 0, the other converges.
    One environment may not serve two members (its intermediate buffers are per problem)."""
    torch, lcc = need_gpu()
    env = chain["env"]
    with pytest.raises(lcc.LccError):
        lcc.Batch(ctx, [env, env])
    env2 = ctx.build_environments(ctx.create_hamiltonian(chain["spec"]), chain["mps"])
    b = to_dev(torch, chain["b"], torch.float64)
    v = to_dev(torch, chain["v"], torch.float64)
    batch = lcc.Batch(ctx, [env, env2])
    xs = [torch.zeros_like(b), torch.zeros_like(b)]
    status, infos = batch.solve([b, torch.zeros_like(b)], [chain["e0"], chain["e0"]], xs, vs=[v, v],
                                precision="fp32", tol=1e-10, max_iter=2000)
    assert status == "LCC_OK"
    assert abs(infos[0]["hylleraas"] - chain["jstar"]) <= 1e-8
    assert infos[1]["iterations"] == 0 and float(xs[1].abs().max()) == 0.0


def test_destroy_order_leaves_no_error():
    """Handles may be destroyed in any order (a garbage collector may finalise a context before
    the environments made on it); later work on a new context is unaffected."""
    torch, lcc = need_gpu()
    spec, mps = C.make("hubbard1d_k8_m64")
    ctx = lcc.Context(0)
    ham = ctx.create_hamiltonian(spec)
    env = ctx.build_environments(ham, mps)
    ctx.close()
    env.close()
    ham.close()
    ctx2 = lcc.Context(0)
    env2 = ctx2.build_environments(ctx2.create_hamiltonian(spec), mps)
    x = to_dev(torch, env2.pack(M.random_two_site_vector(mps, 3)), torch.float64)
    y = torch.empty_like(x)
    env2.apply_heff(x, y, "fp64")
    torch.cuda.synchronize()
    assert torch.isfinite(y).all()
