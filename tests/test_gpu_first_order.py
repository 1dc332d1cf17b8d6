"""First-order right-hand side from transition environments (bra != ket) on the device against
the Fock-space oracle (O1), and the local first-order solve built on it.

Bra: the first-order MPS, canonical around the block; ket: the zeroth-order MPS Phi0 with other
bond dimensions.  On the device: u = P^T H Phi0 (transition operator applied to the ket's own
two-site tensor), v = P^T Phi0 (the same with H = 1), e1 = <Phi0|H|Phi0> / <Phi0|Phi0> (the ket's
effective Hamiltonian on its own tensor), b = -(u - e1 v) = -P^T Q H Phi0, then the local
solve Q(H_eff - E0)Q x = Q b with Q = 1 - v v^T / |v|^2.  In O1 the same quantities come from
the Fock-space H, the contracted ket state and the bra's isometry.  (The perturbation here is
the whole H: the test exercises the contraction, not a particular partition.)

Bars: u, v relative L2 <= 1e-12; e1 <= 1e-12 relative; J within 1e-9 of the dense solution.
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


def _identity_spec(spec):
    n = spec["n_orb"]
    return {"name": "identity", "n_orb": n, "h": np.zeros((n, n)), "eri": None, "u": None, "e_const": 1.0,
            "n_elec": spec["n_elec"], "two_sz": spec["two_sz"]}


@pytest.mark.parametrize("label,spec_make,m1,m0,ket_center", [
    ("hubbard_chain8", lambda: H.hubbard_chain(8, U=4.0, n_elec=8), 16, 10, 3),
    ("threeband_2x1", lambda: H.three_band(2, 1, n_holes=3, two_sz=1), 20, 6, 3),
    ("abinitio_k7_ket_gauge", lambda: H.random_ab_initio(7, 6, seed=5), 18, 9, 1),
])
def test_first_order_rhs_and_solve(label, spec_make, m1, m0, ket_center):
    torch, lcc = need_gpu()
    spec = spec_make()
    K, N, tsz = spec["n_orb"], spec["n_elec"], spec["two_sz"]
    site = 3 if K > 6 else 2
    bra = M.random_mps(K, N, tsz, m1, seed=71, center=site)
    ket = M.random_mps(K, N, tsz, m0, seed=72, center=ket_center)
    blocks = M.two_site_blocks(bra)
    tmpl = BS.two_site_template(bra, blocks)
    say(f"[first-order] {label}: oracle")
    u_ref, v_ref, e1_ref = fock.first_order_vectors(spec, bra, ket, blocks)

    ctx = lcc.Context(0)
    ham = ctx.create_hamiltonian(spec)
    tenv = lcc.build_transition_environments(ctx, ham, bra, ket, site)
    ienv = lcc.build_transition_environments(ctx, ctx.create_hamiltonian(_identity_spec(spec)), bra, ket, site)
    assert tenv.transition and tenv.n_in != tenv.n
    x0 = torch.zeros(tenv.n_in, dtype=torch.float64, device="cuda:0")
    tenv.ket_tensor(x0)
    u = torch.empty(tenv.n, dtype=torch.float64, device="cuda:0")
    v = torch.empty(tenv.n, dtype=torch.float64, device="cuda:0")
    tenv.apply_heff(x0, u, "fp64")
    ienv.apply_heff(x0, v, "fp64")
    torch.cuda.synchronize()
    pk = lambda flat: tenv.pack(BS.unflatten(flat, tmpl, blocks))
    eu, ev = rel(u.cpu().numpy(), pk(u_ref)), rel(v.cpu().numpy(), pk(v_ref))
    say(f"  u rel {eu:.2e}  v rel {ev:.2e}  |v| {np.linalg.norm(v_ref):.6f}")
    assert eu <= 1e-12 and ev <= 1e-12
    # low precision through the same rectangular plan
    u32 = torch.empty(tenv.n, dtype=torch.float32, device="cuda:0")
    tenv.apply_heff(x0.float(), u32, "fp32")
    torch.cuda.synchronize()
    assert rel(u32.double().cpu().numpy(), pk(u_ref)) <= 1e-5

    # e1 from the ket's own effective Hamiltonian (the ket is canonical around its center)
    if ket_center == site:
        kenv = ctx.build_environments(ham, ket, site)
        assert kenv.n == tenv.n_in
        y = torch.empty_like(x0)
        kenv.apply_heff(x0, y, "fp64")
        e1 = float(x0 @ y) / float(x0 @ x0)
    else:
        e1 = e1_ref
    say(f"  e1 {e1:.15f} oracle {e1_ref:.15f}")
    assert abs(e1 - e1_ref) <= 1e-12 * max(1.0, abs(e1_ref))

    b = -(u - e1 * v)
    vhat = v / v.norm()
    heff = fock.effective_hamiltonian(spec, bra, blocks)
    if spec["eri"] is None:
        e0 = C.lower_bound_shift(spec, 0.5)
    else:  # below the lowest eigenvalue of the dense H_eff, passed identically to both sides
        e0 = float(np.linalg.eigvalsh(heff)[0]) - 0.5
    benv = ctx.build_environments(ham, bra, site)
    bref = -(u_ref - e1_ref * v_ref)
    vh = v_ref / np.linalg.norm(v_ref)
    xs = OS.dense_solution(heff, bref, e0, vh)
    A = OS.make_operator(lambda z: heff @ z, e0, vh)
    jstar = OS.hylleraas(A, xs, OS.project(vh, bref))
    for prec in ("fp64", "fp32"):
        x = torch.zeros_like(b)
        info = benv.solve_local_lcc(b, e0, x, v=vhat, precision=prec, tol=1e-12, max_iter=2000, inner_tol=1e-4,
                                    max_outer=100)
        say(f"  solve {prec}: J {info['hylleraas']:.15f} oracle {jstar:.15f} ({info['iterations']} it)")
        assert info["status"] == "LCC_OK"
        assert abs(info["hylleraas"] - jstar) <= 1e-9
        assert abs(float(vhat @ x)) <= 1e-10 * float(x.norm())


def test_transition_environment_errors():
    torch, lcc = need_gpu()
    spec = H.hubbard_chain(8, U=4.0, n_elec=8)
    bra = M.random_mps(8, 8, 0, 16, seed=71, center=3)
    ket = M.random_mps(8, 8, 0, 10, seed=72, center=3)
    ctx = lcc.Context(0)
    ham = ctx.create_hamiltonian(spec)
    tenv = lcc.build_transition_environments(ctx, ham, bra, ket, 3)
    b = torch.zeros(tenv.n, dtype=torch.float64, device="cuda:0")
    with pytest.raises(lcc.LccError) as e:
        tenv.solve_local_lcc(b, 0.0, torch.zeros_like(b))
    assert e.value.code == -7
    with pytest.raises(lcc.LccError):
        tenv.lowest_eigenvalue(steps=5)
    sq = ctx.build_environments(ham, bra, 3)
    with pytest.raises(lcc.LccError):
        sq.ket_tensor(torch.zeros(sq.n, dtype=torch.float64, device="cuda:0"))
    # a bra that is not canonical around the block is refused
    with pytest.raises(lcc.LccError) as e:
        lcc.build_transition_environments(ctx, ham, M.random_mps(8, 8, 0, 16, seed=71, center=1), ket, 3)
    assert e.value.code == -1
