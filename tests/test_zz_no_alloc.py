"""lcc_lowest_eigenvalue_noalloc (Krylov basis in the library's fixed per-device array, no
device allocation) against lcc_lowest_eigenvalue (the same Lanczos cycle on memory allocated per
call): identical Ritz value and residual on consecutive calls whose vector lengths shrink and
then grow again, so that contents left in the array by an earlier call cannot leak into a later
result; sizes beyond the array are refused."""
import pytest

from gpu_common import need_gpu, say
from workloads import configs as C
from workloads import hamiltonians as H
from workloads import mps as M

pytestmark = pytest.mark.gpu


def test_noalloc_matches_allocating_entry_point():
    torch, lcc = need_gpu()
    ctx = lcc.Context(0)
    spec1, mps1 = C.make("hubbard1d_k8_m64")
    env1 = ctx.build_environments(ctx.create_hamiltonian(spec1), mps1)
    spec2 = H.random_ab_initio(8, 6, seed=31)
    mps2 = M.random_mps(8, 6, 0, 20, seed=32)
    env2 = ctx.build_environments(ctx.create_hamiltonian(spec2), mps2)
    assert env2.n < env1.n
    for label, env, steps, seed in (("chain8", env1, 60, 9), ("abinitio_k8", env2, 40, 4), ("chain8 again", env1, 30, 5)):
        ref = env.lowest_eigenvalue(steps=steps, seed=seed)
        got = env.lowest_eigenvalue_noalloc(steps=steps, seed=seed)
        say(f"[noalloc] {label} n={env.n} steps={steps}: {got} vs {ref}")
        assert abs(got[0] - ref[0]) <= 1e-12 * max(1.0, abs(ref[0]))
        assert abs(got[1] - ref[1]) <= 1e-9 * max(1.0, abs(ref[0]))


def test_noalloc_refuses_sizes_beyond_the_array():
    torch, lcc = need_gpu()
    ctx = lcc.Context(0)
    spec, mps = C.make("hubbard2d_4x4_m500")
    env = ctx.build_environments(ctx.create_hamiltonian(spec), mps)
    assert (40 + 2) * env.n * 8 > 64 << 20  # the basis of 40 steps does not fit
    with pytest.raises(lcc.LccError) as e:
        env.lowest_eigenvalue_noalloc(steps=40, seed=1)
    assert e.value.code == -1
    with pytest.raises(lcc.LccError):
        env.lowest_eigenvalue_noalloc(steps=0, seed=1)
    with pytest.raises(lcc.LccError):
        env.lowest_eigenvalue_noalloc(steps=129, seed=1)
    ref = env.lowest_eigenvalue(steps=20, seed=3)
    got = env.lowest_eigenvalue_noalloc(steps=20, seed=3)
    say(f"[noalloc] 4x4 M=500 n={env.n} steps=20: {got} vs {ref}")
    assert abs(got[0] - ref[0]) <= 1e-12 * max(1.0, abs(ref[0]))
