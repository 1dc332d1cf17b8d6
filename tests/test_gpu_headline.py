"""The benchmarked workload (ab initio, 24 orbitals, 12 electrons, M = 1000, two-site block at the
chain centre) against the oracle's full-size results (tests/golden/abinitio_k24_m1000.json, written
by tests/golden/make_abinitio_k24_m1000.py from oracle/ only: the oracle's own two-sided MPO and
its block-sparse contraction).

* H_eff x for the seeded x: 2048 sampled entries (relative L2 over the sample), ||y|| and <z, y>
  for a second seeded vector, under the default plan and under the plan the benchmark runs (the
  shipped tuning cache), in FP64 (<= 1e-12), FP32 (<= 1e-5) and BF16x3 (<= 1e-4).
* The local solve (H_eff - E0) x = b with the oracle's E0 and the benchmark's b, FP64 and mixed
  precision: |J - J*| <= 1e-8 and sampled entries of x within 1e-6 (relative L2).
"""
import json
import os

import numpy as np
import pytest

from gpu_common import need_gpu, say, to_dev
from workloads import configs as C
from workloads import mps as M

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden", "abinitio_k24_m1000.json")


def _flat_index(env, samples):
    idx, val = [], []
    for ia, s1, s2, ib, i, j, v in samples:
        off, ld, rows, cols = env.blocks[(ia, s1, s2, ib)]
        assert i < rows and j < cols
        idx.append(off + i * ld + j)
        val.append(v)
    return np.array(idx), np.array(val)


@pytest.fixture(scope="module")
def headline():
    if not os.path.exists(GOLD):
        pytest.skip("oracle results of the headline workload not generated")
    torch, lcc = need_gpu()
    gold = json.load(open(GOLD))
    spec, mps = C.make("abinitio_k24_m1000")
    say("[headline] K=24 M=1000: environments (default plan)")
    ctx = lcc.Context(0)
    env = ctx.build_environments(ctx.create_hamiltonian(spec), mps)
    assert env.n == gold["n"]
    say("[headline] environments (benchmarked plan from the shipped tuning cache)")
    tctx = lcc.Context(0)
    tctx.set_tune_cache(os.path.join(os.path.dirname(lcc.LIB_PATH), "tune_cache.txt"))
    tenv = tctx.build_environments(tctx.create_hamiltonian(spec), mps)
    return gold, mps, env, tenv


@pytest.mark.parametrize("plan", ["default", "benchmarked"])
def test_apply_vs_oracle(headline, plan):
    torch, lcc = need_gpu()
    gold, mps, env0, tenv = headline
    env = env0 if plan == "default" else tenv
    x = to_dev(torch, env.pack(M.random_two_site_vector(mps, gold["apply"]["x_seed"])), torch.float64)
    z = env.pack(M.random_two_site_vector(mps, gold["apply"]["z_seed"]))
    idx, ref = _flat_index(env, gold["apply"]["samples"])
    for prec, tol in (("fp64", 1e-12), ("fp32", 1e-5), ("bf16x3", 1e-4)):
        xx = x if prec == "fp64" else x.float()
        y = torch.empty_like(xx)
        env.apply_heff(xx, y, prec)
        torch.cuda.synchronize()
        yh = y.double().cpu().numpy()
        e_s = np.linalg.norm(yh[idx] - ref) / np.linalg.norm(ref)
        e_n = abs(np.linalg.norm(yh) - gold["apply"]["norm_y"]) / gold["apply"]["norm_y"]
        e_z = abs(z @ yh - gold["apply"]["z_dot_y"]) / gold["apply"]["norm_y"]
        say(f"[headline] {plan} {prec}: sampled rel L2 {e_s:.2e}, |y| rel {e_n:.2e}, <z,y> rel {e_z:.2e}")
        assert e_s <= tol and e_n <= tol and e_z <= tol


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3"])
def test_solve_vs_oracle(headline, precision):
    torch, lcc = need_gpu()
    gold, mps, _, env = headline
    sol = gold["solve"]
    e0 = gold["shift"]["e0"]
    b = to_dev(torch, env.pack(M.random_two_site_vector(mps, sol["b_seed"])), torch.float64)
    x = torch.zeros_like(b)
    info = env.solve_local_lcc(b, e0, x, precision=precision, tol=1e-10, max_iter=5000, inner_tol=1e-4,
                               max_outer=200)
    idx, ref = _flat_index(env, sol["samples_x"])
    e_x = np.linalg.norm(x.cpu().numpy()[idx] - ref) / np.linalg.norm(ref)
    say(f"[headline] solve {precision}: J {info['hylleraas']:.15f} oracle J* {sol['hylleraas']:.15f} "
        f"(|dJ| {abs(info['hylleraas'] - sol['hylleraas']):.2e}), x sampled rel {e_x:.2e}, {info['iterations']} it")
    assert info["status"] == "LCC_OK"
    assert abs(info["hylleraas"] - sol["hylleraas"]) <= 1e-8
    assert e_x <= 1e-6
