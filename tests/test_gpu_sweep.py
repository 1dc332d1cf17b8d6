"""Two-site sweep (local solve -> SVD split per middle sector -> truncation -> device update of
the left environment -> next guess) against the oracle's sweep, step by step.

Singular vectors carry a free sign (and a free rotation inside a degenerate multiplet), so
only gauge-invariant results are compared: the local energy J* of every block, the
singular values of every split, the number of kept states and the discarded weight.  The
right-hand side of each later block is the normalised guess produced by the previous split
on each side, so an error in the split, the truncation, the left-environment update or the guess
contraction changes the next J*.
"""
import numpy as np
import pytest

from gpu_common import need_gpu, say, to_dev
from oracle import mpo as OM
from oracle import sweep as OW
from workloads import configs as C
from workloads import mps as M

pytestmark = pytest.mark.gpu


def _oracle_sweep(spec, mps, b0, e0, steps, m_max):
    mpo = OM.build_mpo(spec)
    out = []
    b = b0
    for _ in range(steps):
        x, jstar, _ = OW.local_solve(spec, mps, mpo, b, e0)
        if mps["center"] + 2 >= mps["n_sites"]:  # the last block: nothing to split
            out.append({"site": mps["center"], "J": jstar})
            break
        site_blocks, new_bond, guess, sv = OW.split(x, mps, m_max)
        kept = sum(d for _, _, d in new_bond)
        w = sv ** 2
        out.append({"site": mps["center"], "J": jstar, "sv": sv, "kept": kept,
                    "discarded": float(w[kept:].sum() / w.sum())})
        mps = OW.advance(mps, site_blocks, new_bond)
        nrm = np.sqrt(sum(float((g * g).sum()) for g in guess.values()))
        b = {k: g / nrm for k, g in guess.items()}
    return out


@pytest.mark.parametrize("name,m,first,steps,m_max,seed,plan", [
    ("hubbard2d_4x4_m500", 48, 5, 4, 30, 21, 0),       # truncating sweep across the middle
    ("threeband_4x2_m2000", 40, 2, 3, 1000, 22, 0),    # m_max above every bond: nothing discarded
    ("hubbard2d_4x4_m500", 48, 5, 4, 30, 23, 1),       # environments planned as the benchmark plans them
])
def test_sweep_matches_oracle(name, m, first, steps, m_max, seed, plan):
    torch, lcc = need_gpu()
    spec, mps = C.make(name, m_max=m, seed=seed, center=first)
    e0 = C.lower_bound_shift(spec, 0.5)
    b0 = M.random_two_site_vector(mps, seed + 1)
    say(f"[sweep] {name} M={m} first={first} steps={steps} m_max={m_max}: oracle")
    ref = _oracle_sweep(spec, mps, b0, e0, steps, m_max)
    ctx = lcc.Context(0)
    if plan:  # column-major intermediate, channel-major phase 2, large tiles, short split-K parts
        ctx.set_plan(8192.0, 1024, 1, 1)
    ham = ctx.create_hamiltonian(spec)
    sw = lcc.Sweep(ctx, ham, mps, first)
    env = sw.env()
    b = to_dev(torch, env.pack(b0), torch.float64)
    for k, r in enumerate(ref):
        x = torch.zeros_like(b)
        info = env.solve_local_lcc(b, e0, x, precision="fp64", tol=1e-12, max_iter=4000)
        say(f"  block {first + k}: J gpu {info['hylleraas']:.15f} oracle {r['J']:.15f} ({info['iterations']} it)")
        assert info["status"] == "LCC_OK"
        assert abs(info["hylleraas"] - r["J"]) <= 1e-9
        split = sw.advance(x, m_max)
        sv = sw.singular_values()
        say(f"    kept {split['kept']} / {split['n_singular']} (oracle {r['kept']}), "
            f"discarded {split['discarded_weight']:.3e} (oracle {r['discarded']:.3e})")
        assert split["site"] == first + k
        assert split["kept"] == r["kept"]
        assert split["n_singular"] == len(r["sv"])
        np.testing.assert_allclose(sv, r["sv"], rtol=0, atol=1e-9 * r["sv"][0])
        assert abs(split["discarded_weight"] - r["discarded"]) <= 1e-9
        env = sw.env()
        b = torch.empty(env.n, dtype=torch.float64, device="cuda:0")
        sw.guess(b)
        b /= b.norm()
    sw.close()


def test_sweep_errors():
    torch, lcc = need_gpu()
    spec, mps = C.make("hubbard1d_k8_m64", center=5)
    ctx = lcc.Context(0)
    ham = ctx.create_hamiltonian(spec)
    with pytest.raises(lcc.LccError):
        lcc.Sweep(ctx, ham, mps, 7)  # no block starts at the last site
    sw = lcc.Sweep(ctx, ham, mps, 5)
    env = sw.env()
    x = to_dev(torch, env.pack(M.random_two_site_vector(mps, 3)), torch.float64)
    with pytest.raises(lcc.LccError):
        sw.advance(x, 0)  # m_max must be positive
    sw.advance(x, 64)
    env = sw.env()
    x = torch.zeros(env.n, dtype=torch.float64, device="cuda:0")
    sw.guess(x)
    assert float(x.norm()) > 0
    with pytest.raises(lcc.LccError):
        sw.advance(x, 64)  # block (6, 7) is the last one
    sw.close()


def test_sweep_across_both_boundaries():
    """Complete-basis chain (K=8): every block from the left end (0,1) to the right end (6,7),
    against the oracle, then the advance past the last block is refused."""
    torch, lcc = need_gpu()
    spec, mps = C.make("hubbard1d_k8_m64", center=0)
    e0 = C.lower_bound_shift(spec, 0.5)
    b0 = M.random_two_site_vector(mps, 41)
    ref = _oracle_sweep(spec, mps, b0, e0, 7, 64)
    ctx = lcc.Context(0)
    sw = lcc.Sweep(ctx, ctx.create_hamiltonian(spec), mps, 0)
    env = sw.env()
    b = to_dev(torch, env.pack(b0), torch.float64)
    for k, r in enumerate(ref):
        x = torch.zeros_like(b)
        info = env.solve_local_lcc(b, e0, x, precision="fp64", tol=1e-12, max_iter=4000)
        assert abs(info["hylleraas"] - r["J"]) <= 1e-9, k
        if k == 6:
            with pytest.raises(lcc.LccError):
                sw.advance(x, 64)
            break
        split = sw.advance(x, 64)
        assert split["kept"] == r["kept"] and split["n_singular"] == len(r["sv"])
        np.testing.assert_allclose(sw.singular_values(), r["sv"], rtol=0, atol=1e-9 * r["sv"][0])
        env = sw.env()
        b = torch.empty(env.n, dtype=torch.float64, device="cuda:0")
        sw.guess(b)
        b /= b.norm()
    sw.close()


def test_rank_deficient_split():
    """A two-site tensor with a single non-zero block: all other singular values are zero and
    are never kept; the split keeps exactly the rank, like the oracle."""
    torch, lcc = need_gpu()
    spec, mps = C.make("hubbard2d_4x4_m500", m_max=40, seed=51, center=6)
    full = M.random_two_site_vector(mps, 52)
    key = max(full, key=lambda k: full[k].size)
    x = {key: full[key]}
    _, _, _, sv = OW.split(x, mps, 1000)
    ctx = lcc.Context(0)
    sw = lcc.Sweep(ctx, ctx.create_hamiltonian(spec), mps, 6)
    env = sw.env()
    xd = to_dev(torch, env.pack(x), torch.float64)
    split = sw.advance(xd, 1000)
    rank = int(np.linalg.matrix_rank(full[key]))
    say(f"[sweep] rank-deficient block {key}: rank {rank}, kept {split['kept']} / {split['n_singular']}")
    assert split["kept"] == rank
    np.testing.assert_allclose(sw.singular_values(), sv, rtol=0, atol=1e-12 * sv[0])
    # the guess carries the whole norm of x (nothing was discarded)
    env = sw.env()
    g = torch.empty(env.n, dtype=torch.float64, device="cuda:0")
    sw.guess(g)
    assert abs(float(g.norm()) - np.linalg.norm(full[key])) <= 1e-12 * np.linalg.norm(full[key])
    assert split["discarded_weight"] == 0.0
    sw.close()
