"""Batched local solves (one merged launch per GEMM phase, device-side CG scalars and flags,
graph-replayed iterations) against the oracle and against the single-problem solver.

Every member must reach the oracle's Hylleraas energy within 1e-8; the batch is solved
twice in a row with different right-hand sides and precisions (the captured iteration is
replayed many times per solve, with the program's own eager work in between), and a
channel-chunked environment (small intermediate limit) must give the same answer as an
unchunked one.
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


def _oracle_problem(spec, mps, e0, seed, v=None):
    blocks = M.two_site_blocks(mps)
    tmpl = BS.two_site_template(mps, blocks)
    oenv = BS.Environments(spec, mps, OM.build_mpo(spec))
    ap = lambda z: BS.flatten(oenv.apply(BS.unflatten(z, tmpl, blocks)), blocks)
    b = M.random_two_site_vector(mps, seed)
    bflat = BS.flatten(b, blocks)
    A = OS.make_operator(ap, e0, v)
    xo, _, _, _ = OS.cg(A, bflat, tol=1e-13, max_iter=4000, v=v)
    return b, OS.hylleraas(A, xo, OS.project(v, bflat)), xo, tmpl, blocks


@pytest.fixture(scope="module")
def problems():
    torch, lcc = need_gpu()
    ctx = lcc.Context(0)
    out = []
    # complete-basis chain with the ground-state projector (singular but consistent)
    spec, mps = C.make("hubbard1d_k8_m64")
    blocks = M.two_site_blocks(mps)
    heff = fock.effective_hamiltonian(spec, mps, blocks)
    w, U = np.linalg.eigh(heff)
    out.append(("chain8", spec, mps, w[0], U[:, 0]))
    for name, m, seed in [("hubbard2d_4x4_m500", 60, 11), ("threeband_4x2_m2000", 120, 12),
                          ("hubbard2d_4x4_m500", 90, 13)]:
        spec, mps = C.make_member(name, m, seed)
        out.append((f"{name}@{m}", spec, mps, C.lower_bound_shift(spec, 0.5), None))
    spec = H.random_ab_initio(10, 6, seed=61)
    mps = M.random_mps(10, 6, 0, 30, seed=62)
    oenv = BS.Environments(spec, mps, OM.build_mpo(spec))
    bl = M.two_site_blocks(mps)
    tm = BS.two_site_template(mps, bl)
    n = sum(v.size for v in tm.values())
    th, res, _ = OS.lanczos_lowest(lambda z: BS.flatten(oenv.apply(BS.unflatten(z, tm, bl)), bl), n, steps=120)
    out.append(("abinitio_k10", spec, mps, th - max(0.5, 2 * res), None))
    envs, refs = [], []
    for i, (label, spec, mps, e0, v) in enumerate(out):
        say(f"[batch] member {label}: environments + oracle")
        env = ctx.build_environments(ctx.create_hamiltonian(spec), mps)
        envs.append(env)
        refs.append((label, spec, mps, e0, v))
    return ctx, envs, refs


@pytest.mark.parametrize("precision,seed", [("fp32", 100), ("bf16x3", 200)])
def test_batch_matches_oracle_and_single(problems, precision, seed):
    torch, lcc = need_gpu()
    ctx, envs, refs = problems
    batch = lcc.Batch(ctx, envs)
    bs, xs, vs, e0s, exp = [], [], [], [], []
    for i, ((label, spec, mps, e0, v), env) in enumerate(zip(refs, envs)):
        vflat = None
        if v is not None:
            blocks = M.two_site_blocks(mps)
            vflat = v
        b, jstar, xo, tmpl, blocks = _oracle_problem(spec, mps, e0, seed + i, vflat)
        bs.append(to_dev(torch, env.pack(b), torch.float64))
        xs.append(torch.zeros_like(bs[-1]))
        vs.append(None if v is None else to_dev(torch, env.pack(BS.unflatten(v, tmpl, blocks)), torch.float64))
        e0s.append(e0)
        exp.append((label, jstar, env.pack(BS.unflatten(xo, tmpl, blocks))))
    say(f"[batch] solve {precision}")
    status, infos = batch.solve(bs, e0s, xs, vs=vs, precision=precision, tol=1e-10, max_iter=4000)
    assert status == "LCC_OK", (status, infos)
    for (label, jstar, xref), info, x in zip(exp, infos, xs):
        say(f"  {label}: {info}")
        assert abs(info["hylleraas"] - jstar) <= 1e-8, label
        assert info["rel_residual"] <= 1e-10
        assert rel(x.cpu().numpy(), xref) <= 1e-6, label
    # the single-problem solver on the same inputs agrees
    for (label, jstar, _), env, b, v, e0 in zip(exp, envs, bs, vs, e0s):
        x1 = torch.zeros_like(b)
        one = env.solve_local_lcc(b, e0, x1, v=v, precision=precision)
        assert abs(one["hylleraas"] - jstar) <= 1e-8, label


def test_chunked_intermediate_matches(problems):
    torch, lcc = need_gpu()
    ctx, envs, refs = problems
    label, spec, mps, e0, v = refs[2]
    ctx2 = lcc.Context(0)
    ctx2.set_intermediate_limit(64 * 1024)  # forces many channel chunks
    env_c = ctx2.build_environments(ctx2.create_hamiltonian(spec), mps)
    env_u = envs[2]
    x = to_dev(torch, env_u.pack(M.random_two_site_vector(mps, 9)), torch.float64)
    y1 = torch.empty_like(x)
    y2 = torch.empty_like(x)
    env_u.apply_heff(x, y1, "fp64")
    env_c.apply_heff(x, y2, "fp64")
    torch.cuda.synchronize()
    say(f"[batch] chunked vs unchunked: {rel(y2.cpu().numpy(), y1.cpu().numpy()):.2e}")
    assert rel(y2.cpu().numpy(), y1.cpu().numpy()) <= 1e-13
    assert env_c.flops_per_apply == env_u.flops_per_apply


def test_batch_members_with_different_plans(problems):
    """Members planned with different operand layouts (row- and column-major intermediate, as
    tuning-cache entries of different histograms can choose) are merged per layout, so every
    member keeps its own transposition."""
    torch, lcc = need_gpu()
    _, _, refs = problems
    pctx = lcc.Context(0)
    members = []
    for i, idx in enumerate((1, 2, 4, 1)):
        label, spec, mps, e0, v = refs[idx]
        if i % 2:
            pctx.set_plan(8192.0, 1024, 1, 1)
        else:
            pctx.set_plan(2048.0, 2048, 0, 0)
        members.append((f"{label} plan {i % 2}", spec, mps, e0, pctx.build_environments(pctx.create_hamiltonian(spec), mps)))
    batch = lcc.Batch(pctx, [m[4] for m in members])
    bs, xs, e0s, exp = [], [], [], []
    for i, (label, spec, mps, e0, env) in enumerate(members):
        b, jstar, _, _, _ = _oracle_problem(spec, mps, e0, 300 + i)
        bs.append(to_dev(torch, env.pack(b), torch.float64))
        xs.append(torch.zeros_like(bs[-1]))
        e0s.append(e0)
        exp.append((label, jstar))
    status, infos = batch.solve(bs, e0s, xs, precision="fp32", tol=1e-10, max_iter=4000, inner_tol=1e-4)
    assert status == "LCC_OK", (status, infos)
    for (label, jstar), info in zip(exp, infos):
        say(f"  {label}: J {info['hylleraas']:.12f} vs {jstar:.12f}")
        assert abs(info["hylleraas"] - jstar) <= 1e-8, label


def test_one_shot_batched_entry_point(problems):
    """lcc_solve_local_lcc_batched (create, solve, destroy in one call) on three members,
    against the oracle's J*."""
    torch, lcc = need_gpu()
    ctx, envs, refs = problems
    sel = (1, 2, 4)
    bs, xs, e0s, exp = [], [], [], []
    for k, i in enumerate(sel):
        label, spec, mps, e0, v = refs[i]
        b, jstar, _, _, _ = _oracle_problem(spec, mps, e0, 500 + k)
        bs.append(to_dev(torch, envs[i].pack(b), torch.float64))
        xs.append(torch.zeros_like(bs[-1]))
        e0s.append(e0)
        exp.append((label, jstar))
    status, infos = lcc.solve_local_lcc_batched([envs[i] for i in sel], bs, e0s, xs, precision="fp32", tol=1e-10,
                                                max_iter=4000, inner_tol=1e-4)
    assert status == "LCC_OK", (status, infos)
    for (label, jstar), info in zip(exp, infos):
        say(f"  one-shot {label}: J {info['hylleraas']:.12f} vs {jstar:.12f}")
        assert abs(info["hylleraas"] - jstar) <= 1e-8, label
    # a repeated environment is refused
    with pytest.raises(lcc.LccError):
        lcc.solve_local_lcc_batched([envs[1], envs[1]], bs[:1] * 2, e0s[:1] * 2, [torch.zeros_like(bs[0]) for _ in range(2)])
