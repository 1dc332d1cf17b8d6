"""Autotuner: every candidate plan and kernel choice computes the same H_eff x (to rounding),
the tuned plan matches the oracle, and the tuning cache reproduces the choice for a new
environment with the same block-size histogram without timing anything."""
import numpy as np
import pytest

from gpu_common import need_gpu, rel, say, to_dev
from oracle import blocksparse as BS
from oracle import mpo as OM
from workloads import configs as C
from workloads import mps as M

pytestmark = pytest.mark.gpu


def _oracle_apply(spec, mps, x):
    blocks = M.two_site_blocks(mps)
    oenv = BS.Environments(spec, mps, OM.build_mpo(spec))
    return oenv.apply(x)


def test_autotune_keeps_results_and_caches(tmp_path):
    torch, lcc = need_gpu()
    spec, mps = C.make_member("hubbard2d_4x4_m500", 90, 31)
    x = M.random_two_site_vector(mps, 32)
    ctx = lcc.Context(0)
    cache = tmp_path / "tune.txt"
    ctx.set_tune_cache(cache)
    env = ctx.build_environments(ctx.create_hamiltonian(spec), mps)
    ref = env.pack(_oracle_apply(spec, mps, x))
    xd = to_dev(torch, env.pack(x), torch.float64)
    y = torch.empty_like(xd)
    env.apply_heff(xd, y, "fp64")
    torch.cuda.synchronize()
    assert rel(y.cpu().numpy(), ref) <= 1e-12
    info = env.autotune("fp32", reps=2)
    say(f"[tune] {info}")
    assert info["candidates"] == 54 and not info["from_cache"]
    assert 0 <= info["packed_launches"] <= info["launches"]
    for prec, tol in (("fp64", 1e-12), ("fp32", 1e-5), ("bf16x3", 1e-4)):
        xx = xd if prec == "fp64" else xd.float()
        yy = torch.empty_like(xx)
        env.apply_heff(xx, yy, prec)
        torch.cuda.synchronize()
        err = rel(yy.double().cpu().numpy(), ref)
        say(f"  tuned {prec}: rel err vs oracle {err:.2e}")
        assert err <= tol
    lines = cache.read_text().strip().splitlines()
    assert len(lines) == 1
    # a new context with the cache: the environment is planned from the entry
    ctx2 = lcc.Context(0)
    ctx2.set_tune_cache(cache)
    env2 = ctx2.build_environments(ctx2.create_hamiltonian(spec), mps)
    info2 = env2.autotune("fp32", reps=1)
    assert info2["from_cache"] and info2["candidates"] == 0
    keys = ("tile_overhead", "split_k", "p2_order", "t_colmajor")
    assert [info2[k] for k in keys] == [info[k] for k in keys]
    assert info2["packed_launches"] == info["packed_launches"]
    y2 = torch.empty_like(xd)
    env2.apply_heff(xd, y2, "fp64")
    torch.cuda.synchronize()
    assert rel(y2.cpu().numpy(), ref) <= 1e-12
    assert len(cache.read_text().strip().splitlines()) == 1


def test_autotune_rejects_bad_arguments():
    torch, lcc = need_gpu()
    spec, mps = C.make("hubbard1d_k8_m64")
    ctx = lcc.Context(0)
    env = ctx.build_environments(ctx.create_hamiltonian(spec), mps)
    with pytest.raises(lcc.LccError):
        env.autotune("fp32", reps=0)


def test_concurrent_phase_launches_are_bitwise_identical():
    """Launches of one phase write disjoint outputs, so running them on side streams changes
    nothing: y is bitwise the same for every overlap setting and precision."""
    torch, lcc = need_gpu()
    spec, mps = C.make_member("threeband_4x2_m2000", 150, 33)
    ctx = lcc.Context(0)
    env = ctx.build_environments(ctx.create_hamiltonian(spec), mps)
    x64 = to_dev(torch, env.pack(M.random_two_site_vector(mps, 34)), torch.float64)
    for prec in ("fp64", "fp32", "bf16x3"):
        xx = x64 if prec == "fp64" else x64.float()
        outs = []
        for ov in (0, 3, 1):
            ctx.set_overlap(ov)
            yy = torch.empty_like(xx)
            env.apply_heff(xx, yy, prec)
            torch.cuda.synchronize()
            outs.append(yy)
        assert torch.equal(outs[0], outs[1]) and torch.equal(outs[0], outs[2]), prec
    with pytest.raises(lcc.LccError):
        ctx.set_overlap(-1)


@pytest.mark.parametrize("p2_order,t_colmajor,split_k", [(0, 1, 2048), (1, 1, 512), (1, 0, 1024), (0, 2, 1024),
                                                           (1, 2, 512)])
def test_every_plan_option_matches_oracle(p2_order, t_colmajor, split_k):
    """Planner options (phase-2 order, operator order and intermediate layout, split-K length)
    reorder and re-lay-out the same block products: every combination reproduces the oracle."""
    torch, lcc = need_gpu()
    for name, m, seed in (("hubbard2d_4x4_m500", 70, 41), ("threeband_4x2_m2000", 110, 42)):
        spec, mps = C.make_member(name, m, seed)
        x = M.random_two_site_vector(mps, seed + 1)
        ctx = lcc.Context(0)
        ctx.set_plan(2048.0, split_k, p2_order, t_colmajor)
        env = ctx.build_environments(ctx.create_hamiltonian(spec), mps)
        ref = env.pack(_oracle_apply(spec, mps, x))
        xd = to_dev(torch, env.pack(x), torch.float64)
        for prec, tol in (("fp64", 1e-12), ("fp32", 1e-5), ("bf16x3", 1e-4)):
            xx = xd if prec == "fp64" else xd.float()
            yy = torch.empty_like(xx)
            env.apply_heff(xx, yy, prec)
            torch.cuda.synchronize()
            assert rel(yy.double().cpu().numpy(), ref) <= tol, (name, prec)
    with pytest.raises(lcc.LccError):
        lcc.Context(0).set_plan(2048.0, 0, 0, 0)
