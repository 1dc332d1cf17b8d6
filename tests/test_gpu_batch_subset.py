"""Eight members of the seeded 64-problem batch at their full bond dimensions (the first eight
4x4 Hubbard and 3-band members, M from 362 to 1469) solved in one batched call
(lcc_solve_local_lcc_batched, mixed precision) against the oracle's energies
(tests/golden/batch_subset.json, written by tests/golden/make_batch_subset.py from oracle/ only).

Bar: |J - J*| <= 1e-8 for every member.
"""
import json
import os

import pytest

from gpu_common import need_gpu, say
from workloads import configs as C
from workloads import mps as M

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden", "batch_subset.json")


def test_batch_subset_full_size_vs_oracle():
    if not os.path.exists(GOLD):
        pytest.skip("oracle results of the batch subset not generated")
    torch, lcc = need_gpu()
    gold = json.load(open(GOLD))["members"]
    ctx = lcc.Context(0)
    ctx.set_intermediate_limit(1 << 30)
    envs, bs, xs, e0s, hams = [], [], [], [], {}
    for rec in gold:
        spec, mps = C.make_member(rec["parent"], rec["m"], rec["seed"])
        if rec["parent"] not in hams:
            hams[rec["parent"]] = ctx.create_hamiltonian(spec)
        env = ctx.build_environments(hams[rec["parent"]], mps)
        assert env.n == rec["n"]
        envs.append(env)
        bs.append(torch.tensor(env.pack(M.random_two_site_vector(mps, rec["b_seed"])), dtype=torch.float64,
                               device="cuda:0"))
        xs.append(torch.zeros_like(bs[-1]))
        e0s.append(rec["e0"])
        say(f"[batch subset] member {rec['index']}: {rec['parent']} M={rec['m']} n={env.n}")
    status, infos = lcc.solve_local_lcc_batched(envs, bs, e0s, xs, precision="fp32", tol=1e-10, max_iter=5000,
                                                inner_tol=1e-4)
    assert status == "LCC_OK", (status, infos)
    for rec, info in zip(gold, infos):
        say(f"  member {rec['index']}: J {info['hylleraas']:.15f} oracle {rec['hylleraas']:.15f}")
        assert abs(info["hylleraas"] - rec["hylleraas"]) <= 1e-8
