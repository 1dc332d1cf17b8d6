"""Lowest eigenpair of H_eff on the device (Lanczos with full re-orthogonalisation,
restarted) against dense diagonalisation in the oracle, and one ground-state sweep (the
DMRG energy functional of the Implementation section: eigenpair -> SVD split -> next block)
against the oracle's sweep, block by block.

Bars: eigenvalue within 1e-10 (absolute, energies of order 10); eigenvector overlap
|<u, u*>| >= 1 - 1e-10 (non-degenerate ground states); sweep energies within 1e-9.
"""
import numpy as np
import pytest

from gpu_common import need_gpu, say, to_dev
from oracle import blocksparse as BS
from oracle import fock
from oracle import mpo as OM
from oracle import sweep as OW
from workloads import configs as C
from workloads import hamiltonians as H
from workloads import mps as M

pytestmark = pytest.mark.gpu


def _poison_device_memory(torch, gib=2):
    # freed pages filled with NaN: buffers the library allocates next may start out as NaN
    t = torch.full((gib << 27,), float("nan"), dtype=torch.float64, device="cuda:0")
    torch.cuda.synchronize()
    del t
    torch.cuda.empty_cache()


@pytest.mark.parametrize("label,make", [
    ("chain8_complete", lambda: C.make("hubbard1d_k8_m64")),
    ("abinitio_k8_m20", lambda: (H.random_ab_initio(8, 6, seed=31), M.random_mps(8, 6, 0, 20, seed=32))),
])
def test_lowest_eigenpair_vs_dense(label, make):
    torch, lcc = need_gpu()
    spec, mps = make()
    blocks = M.two_site_blocks(mps)
    heff = fock.effective_hamiltonian(spec, mps, blocks)
    w, U = np.linalg.eigh(heff)
    tmpl = BS.two_site_template(mps, blocks)
    ctx = lcc.Context(0)
    env = ctx.build_environments(ctx.create_hamiltonian(spec), mps)
    ustar = env.pack(BS.unflatten(U[:, 0], tmpl, blocks))
    _poison_device_memory(torch)
    th, res = env.lowest_eigenvalue(steps=120, seed=5)
    say(f"[eigen] {label} n={env.n}: lanczos theta {th:.14f} res {res:.2e}; dense {w[0]:.14f} (gap {w[1] - w[0]:.3f})")
    assert np.isfinite(th) and np.isfinite(res)
    assert th >= w[0] - 1e-10 and th - w[0] <= max(1e-9, res * res / (w[1] - w[0]) * 10)
    _poison_device_memory(torch)
    x = torch.zeros(env.n, dtype=torch.float64, device="cuda:0")
    info = env.lowest_eigenpair(x, steps=40, max_restarts=40, tol=1e-11, seed=7)
    u = x.cpu().numpy()
    say(f"  eigenpair {info}  overlap {abs(u @ ustar):.15f}")
    assert info["status"] == "LCC_OK"
    assert abs(info["theta"] - w[0]) <= 1e-10
    assert abs(np.linalg.norm(u) - 1.0) <= 1e-12
    assert abs(u @ ustar) >= 1.0 - 1e-10
    # a start vector: the exact eigenvector converges in the first cycle
    x2 = to_dev(torch, ustar, torch.float64)
    info2 = env.lowest_eigenpair(x2, steps=8, max_restarts=1, tol=1e-9, seed=7)
    assert info2["status"] == "LCC_OK" and abs(info2["theta"] - w[0]) <= 1e-10


def test_lowest_eigenpair_errors():
    torch, lcc = need_gpu()
    spec, mps = C.make("hubbard1d_k8_m64")
    ctx = lcc.Context(0)
    env = ctx.build_environments(ctx.create_hamiltonian(spec), mps)
    x = torch.zeros(env.n, dtype=torch.float64, device="cuda:0")
    with pytest.raises(lcc.LccError):
        env.lowest_eigenpair(x, steps=0)
    with pytest.raises(lcc.LccError):
        env.lowest_eigenpair(x, max_restarts=0)
    bad = x.clone()
    bad[3] = float("nan")
    with pytest.raises(lcc.LccError) as e:
        env.lowest_eigenpair(bad)
    assert e.value.code == -4
    # two Krylov vectors, one cycle: reported as not converged, x holds the Ritz vector
    info = env.lowest_eigenpair(x, steps=2, max_restarts=1, tol=1e-12)
    assert info["status"] == "LCC_NOT_CONVERGED"
    assert abs(float(x.norm()) - 1.0) <= 1e-12


def test_ground_state_sweep_matches_oracle():
    """Four blocks of a truncating ground-state sweep of a 3-band Cu-O cluster (2x2 cells, 12
    orbitals, 5 holes; M=20, keep 12): eigenpair on the device, split, next block started from
    the split's guess; the oracle does the same with dense diagonalisation and numpy's SVD."""
    torch, lcc = need_gpu()
    first = 3
    spec = H.three_band(2, 2, n_holes=5, two_sz=1)
    mps = M.random_mps(12, 5, 1, 20, seed=41, center=first)
    mpo = OM.build_mpo(spec)
    m_keep, steps = 12, 4
    ref = []
    om = mps
    for _ in range(steps):
        th, u, gap = OW.local_ground_state(spec, om, mpo)
        site_blocks, new_bond, guess, sv = OW.split(u, om, m_keep)
        ref.append({"theta": th, "gap": gap, "sv": sv, "kept": sum(d for _, _, d in new_bond)})
        om = OW.advance(om, site_blocks, new_bond)
    ctx = lcc.Context(0)
    sw = lcc.Sweep(ctx, ctx.create_hamiltonian(spec), mps, first)
    env = sw.env()
    x = torch.zeros(env.n, dtype=torch.float64, device="cuda:0")
    for k, r in enumerate(ref):
        info = env.lowest_eigenpair(x, steps=40, max_restarts=60, tol=1e-11, seed=3)
        say(f"[dmrg] block {first + k}: theta gpu {info['theta']:.14f} oracle {r['theta']:.14f} gap {r['gap']:.2e}")
        assert info["status"] == "LCC_OK"
        assert abs(info["theta"] - r["theta"]) <= 1e-9
        split = sw.advance(x, m_keep)
        sv = sw.singular_values()
        assert split["kept"] == r["kept"]
        np.testing.assert_allclose(sv, r["sv"], rtol=0, atol=1e-8 * r["sv"][0])
        env = sw.env()
        x = torch.empty(env.n, dtype=torch.float64, device="cuda:0")
        sw.guess(x)
    sw.close()
