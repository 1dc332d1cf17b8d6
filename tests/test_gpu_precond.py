"""diag(H_eff) on the device against the dense Fock-space H_eff (O1), and the Jacobi-preconditioned
local solve (FP64 and mixed precision) against the oracle's exact solution, with and without the
local projector.

Bars: diagonal element-wise within 1e-12 (relative to its largest entry); energies within 1e-9
of J*; the preconditioned solve converges to the same solution as the plain one.
"""
import numpy as np
import pytest

from gpu_common import need_gpu, rel, say, to_dev
from oracle import blocksparse as BS
from oracle import fock
from oracle import solve as OS
from workloads import configs as C
from workloads import hamiltonians as H
from workloads import mps as M

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("label,make", [
    ("chain8_complete", lambda: C.make("hubbard1d_k8_m64")),
    ("abinitio_k8_m20", lambda: (H.random_ab_initio(8, 6, seed=31), M.random_mps(8, 6, 0, 20, seed=32))),
    ("threeband_2x2_offcentre", lambda: (H.three_band(2, 2, n_holes=5, two_sz=1),
                                         M.random_mps(12, 5, 1, 20, seed=41, center=3))),
])
def test_diagonal_and_jacobi_solve(label, make):
    torch, lcc = need_gpu()
    spec, mps = make()
    blocks = M.two_site_blocks(mps)
    tmpl = BS.two_site_template(mps, blocks)
    heff = fock.effective_hamiltonian(spec, mps, blocks)
    ctx = lcc.Context(0)
    env = ctx.build_environments(ctx.create_hamiltonian(spec), mps)
    pk = lambda flat: env.pack(BS.unflatten(flat, tmpl, blocks))
    d = torch.empty(env.n, dtype=torch.float64, device="cuda:0")
    env.diagonal(d)
    dref = pk(np.diag(heff).copy())
    err = np.abs(d.cpu().numpy() - dref).max() / np.abs(dref).max()
    say(f"[precond] {label} n={env.n}: diagonal max rel err {err:.2e}")
    assert err <= 1e-12
    w, U = np.linalg.eigh(heff)
    e0 = w[0] - 0.5
    rng = np.random.Generator(np.random.PCG64(5))
    bflat = rng.standard_normal(heff.shape[0])
    bflat /= np.linalg.norm(bflat)
    b = to_dev(torch, pk(bflat), torch.float64)
    for use_v in (False, True):
        vflat = U[:, 1] if use_v else None  # a projector that leaves the shifted operator definite
        xs = OS.dense_solution(heff, bflat, e0, vflat)
        A = OS.make_operator(lambda z: heff @ z, e0, vflat)
        jstar = OS.hylleraas(A, xs, OS.project(vflat, bflat))
        v = None if vflat is None else to_dev(torch, pk(vflat), torch.float64)
        its = {}
        for prec in ("fp64", "fp32"):
            for pc in ("none", "jacobi"):
                x = torch.zeros_like(b)
                info = env.solve_local_lcc(b, e0, x, v=v, precision=prec, tol=1e-11, max_iter=3000, inner_tol=1e-4,
                                           max_outer=200, preconditioner=pc)
                its[(prec, pc)] = info["iterations"]
                assert info["status"] == "LCC_OK", (prec, pc, info)
                assert abs(info["hylleraas"] - jstar) <= 1e-9, (prec, pc, info["hylleraas"], jstar)
                assert rel(x.cpu().numpy(), pk(xs)) <= 1e-8
        say(f"  projector={use_v}: iterations {its}")


def test_jacobi_refuses_a_shift_above_the_diagonal():
    torch, lcc = need_gpu()
    spec, mps = C.make("hubbard1d_k8_m64")
    ctx = lcc.Context(0)
    env = ctx.build_environments(ctx.create_hamiltonian(spec), mps)
    d = torch.empty(env.n, dtype=torch.float64, device="cuda:0")
    env.diagonal(d)
    b = torch.ones(env.n, dtype=torch.float64, device="cuda:0")
    with pytest.raises(lcc.LccError) as e:
        env.solve_local_lcc(b, float(d.min()) + 1.0, torch.zeros_like(b), preconditioner="jacobi")
    assert e.value.code == -3
