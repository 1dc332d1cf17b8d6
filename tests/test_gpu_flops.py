"""The planner's algorithmic flop count (lcc_env_flops, the work unit of every throughput
figure) against the oracle's exact integer count of the middle-bond factorisation
(oracle.flops.factorised_flops), both for the library's own MPO, on full-size lattice
workloads and the complete-basis chain.  The oracle count is pinned in
test_oracle_flops.py against the work its own contraction performs."""
import pytest

from gpu_common import need_gpu, product_mpo, say
from oracle import flops as OF
from workloads import configs as C
from workloads import hamiltonians as H
from workloads import mps as M

pytestmark = pytest.mark.gpu

CASES = [
    ("hubbard1d_k8_m64", lambda: C.make("hubbard1d_k8_m64")),
    ("hubbard2d_4x4_m500", lambda: C.make("hubbard2d_4x4_m500")),
    ("threeband_4x2_m2000", lambda: C.make("threeband_4x2_m2000")),
    ("abinitio_k10_m60", lambda: (H.random_ab_initio(10, 6, seed=1003), M.random_mps(10, 6, 0, 60, seed=1003))),
]


@pytest.mark.parametrize("order", ["left", "right"])
@pytest.mark.parametrize("label,make", CASES, ids=[c[0] for c in CASES])
def test_planner_flops_equal_oracle_count(label, make, order):
    torch, lcc = need_gpu()
    spec, mps = make()
    ctx = lcc.Context(0)
    ctx.set_plan(2048.0, 2048, 0, 0 if order == "left" else 2)
    ham = ctx.create_hamiltonian(spec)
    say(f"[flops] {label}, {order} operator first: build")
    env = ctx.build_environments(ham, mps)
    f1, f2 = env.flops()
    ref = OF.factorised_flops(mps, product_mpo(ham), order)
    say(f"  planner {f1:.0f} + {f2:.0f}   oracle {ref['left']} + {ref['right']}")
    assert (int(f1), int(f2)) == (ref["left"], ref["right"])
    assert env.flops_per_apply == float(ref["total"])


@pytest.mark.parametrize("order", ["left", "right"])
@pytest.mark.parametrize("name", ["hubbard2d_4x4_m500", "threeband_4x2_m2000"])
def test_one_site_planner_flops_equal_oracle_count(name, order):
    torch, lcc = need_gpu()
    spec, mps = C.make(name)
    m1 = M.canonical_at(mps, mps["center"])
    ctx = lcc.Context(0)
    ctx.set_plan(2048.0, 2048, 0, 0 if order == "left" else 2)
    ham = ctx.create_hamiltonian(spec)
    say(f"[flops] one site, {name}, {order} operator first: build")
    env = ctx.build_environments_one_site(ham, m1, m1["center"])
    f1, f2 = env.flops()
    ref = OF.factorised_flops(m1, product_mpo(ham), order, one_site=True)
    say(f"  planner {f1:.0f} + {f2:.0f}   oracle {ref['left']} + {ref['right']}")
    assert (int(f1), int(f2)) == (ref["left"], ref["right"])
    assert env.flops_per_apply == float(ref["total"])
