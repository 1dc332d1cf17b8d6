"""GPU parity of H_eff x (the HIP path through the C ABI) against the CPU oracle.

Bars: FP64 relative L2 <= 1e-12; raw FP32 <= 1e-5; raw BF16x3 <= 1e-4 (operands split to about 2^-16 relative, FP32 accumulation).
Cases span several tiles and ragged tails (sector dims 1..300), every Hamiltonian family,
the complete-basis chain against exact diagonalisation (O1), and the full-size workloads
either element by element against O2 or, where the oracle cannot hold the environments
(the K = 24 ab initio system at M = 1000), by properties that hold at any size.
"""
import numpy as np
import pytest

from gpu_common import need_gpu, rel, say, to_dev
from oracle import blocksparse as BS
from oracle import fock
from oracle import mpo as OM
from workloads import configs as C
from workloads import hamiltonians as H
from workloads import mps as M

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    torch, lcc = need_gpu()
    return lcc.Context(0)


def _apply(torch, env, xflat, precision):
    dt = torch.float64 if precision == "fp64" else torch.float32
    x = to_dev(torch, xflat, dt)
    y = torch.empty_like(x)
    env.apply_heff(x, y, precision)
    torch.cuda.synchronize()
    return y.double().cpu().numpy()


def _case_o1(ctx, spec, mps, label):
    torch, lcc = need_gpu()
    say(f"[parity-o1] {label}: build")
    ham = ctx.create_hamiltonian(spec)
    env = ctx.build_environments(ham, mps)
    blocks = M.two_site_blocks(mps)
    heff = fock.effective_hamiltonian(spec, mps, blocks)
    x = M.random_two_site_vector(mps, 11)
    yref = heff @ BS.flatten(x, blocks)
    yref_d = BS.unflatten(yref, x, blocks)
    xf = env.pack(x)
    out = {}
    for prec in ("fp64", "fp32", "bf16x3"):
        say(f"[parity-o1] {label}: apply {prec}")
        y = env.unpack(_apply(torch, env, xf, prec))
        out[prec] = rel(BS.flatten(y, blocks), yref)
    return out, env


def test_chain8_complete_basis_vs_ed(ctx):
    spec, mps = C.make("hubbard1d_k8_m64")
    err, env = _case_o1(ctx, spec, mps, "hubbard1d_k8_m64")
    say(f"  errors {err}")
    assert env.n == 4900
    assert err["fp64"] <= 1e-12
    assert err["fp32"] <= 1e-5
    assert err["bf16x3"] <= 1e-4


@pytest.mark.parametrize("label,make,m,seed", [
    ("abinitio_k6", lambda: H.random_ab_initio(6, 6, seed=21), 12, 22),
    ("abinitio_k7_sz1", lambda: H.random_ab_initio(7, 5, two_sz=1, seed=31), 20, 32),
    ("threeband_2x1", lambda: H.three_band(2, 1, n_holes=5, two_sz=1), 24, 41),
    ("rotated_hubbard_k6", lambda: H.rotate_orbitals(H.hubbard_chain(6, U=3.0, n_elec=6), H.random_orthogonal(6, 5)), 16, 51),
])
def test_small_systems_vs_fock(ctx, label, make, m, seed):
    spec = make()
    mps = M.random_mps(spec["n_orb"], spec["n_elec"], spec["two_sz"], m, seed)
    err, _ = _case_o1(ctx, spec, mps, label)
    say(f"  errors {err}")
    assert err["fp64"] <= 1e-12
    assert err["fp32"] <= 1e-5
    assert err["bf16x3"] <= 1e-4


@pytest.mark.parametrize("plan", ["default", "benchmarked"])
def test_every_block_position_vs_fock(plan):
    """The two-site block at every position of the chain, both ends included (one environment
    is the trivial one there), against the Fock-space effective Hamiltonian; with the default
    planner parameters and with those of the benchmarked plan (column-major intermediate,
    channel-major phase 2, large tiles, short split-K parts)."""
    torch, lcc = need_gpu()
    spec = H.random_ab_initio(6, 6, seed=71)
    pctx = lcc.Context(0)
    if plan == "benchmarked":
        pctx.set_plan(8192.0, 1024, 1, 1)
    for center in range(spec["n_orb"] - 1):
        mps = M.random_mps(6, 6, 0, 14, seed=72 + center, center=center)
        err, env = _case_o1(pctx, spec, mps, f"abinitio_k6 block ({center},{center + 1}) {plan}")
        say(f"  n={env.n} errors {err}")
        assert err["fp64"] <= 1e-12, center
        assert err["fp32"] <= 1e-5, center
        assert err["bf16x3"] <= 1e-4, center


def _case_o2(ctx, spec, mps, label, precisions=("fp64", "fp32", "bf16x3")):
    torch, lcc = need_gpu()
    say(f"[parity-o2] {label}: build")
    ham = ctx.create_hamiltonian(spec)
    env = ctx.build_environments(ham, mps)
    oenv = BS.Environments(spec, mps, OM.build_mpo(spec))
    x = M.random_two_site_vector(mps, 13)
    yref = env.pack(oenv.apply(x))
    xf = env.pack(x)
    out = {}
    for prec in precisions:
        say(f"[parity-o2] {label}: apply {prec}")
        out[prec] = rel(_apply(torch, env, xf, prec), yref)
    return out, env


@pytest.mark.parametrize("name,m", [
    ("hubbard2d_4x4_m500", 60),
    ("hubbard2d_4x4_m500", 500),      # full size
    ("threeband_4x2_m2000", 150),
    ("threeband_4x2_m2000", 2000),    # full size
])
def test_lattice_workloads_vs_blocksparse(ctx, name, m):
    spec, mps = C.make(name, m_max=m)
    err, env = _case_o2(ctx, spec, mps, f"{name}@M={m}")
    say(f"  n={env.n} D={env.mpo_bond_dim} errors {err}")
    assert err["fp64"] <= 1e-12
    assert err["fp32"] <= 1e-5
    assert err["bf16x3"] <= 1e-4


def test_abinitio_k10_vs_blocksparse(ctx):
    spec = H.random_ab_initio(10, 6, seed=61)
    mps = M.random_mps(10, 6, 0, 30, seed=62)
    err, env = _case_o2(ctx, spec, mps, "abinitio_k10_m30")
    say(f"  n={env.n} D={env.mpo_bond_dim} errors {err}")
    assert err["fp64"] <= 1e-12
    assert err["fp32"] <= 1e-5


def test_number_operator_full_size(ctx):
    # H = N-hat through the same kernels at the largest workload shape: H_eff x = N x
    torch, lcc = need_gpu()
    spec, mps = C.make("threeband_4x2_m2000")
    nspec = H.number_operator(spec["n_orb"], spec["n_elec"], spec["two_sz"])
    say("[property] number operator, 3-band M=2000: build")
    env = ctx.build_environments(ctx.create_hamiltonian(nspec), mps)
    x = M.random_two_site_vector(mps, 3)
    xf = env.pack(x)
    y = _apply(torch, env, xf, "fp64")
    assert rel(y, spec["n_elec"] * xf) <= 1e-12


def test_abinitio_full_size_hermitian_and_bounded(ctx):
    # K = 24, M = 1000: beyond the oracle's memory; check symmetry <y, A x> = <A y, x> and
    # agreement of the three precisions on the same input
    torch, lcc = need_gpu()
    spec, mps = C.make("abinitio_k24_m1000")
    say("[property] abinitio K=24 M=1000: build")
    env = ctx.build_environments(ctx.create_hamiltonian(spec), mps)
    say(f"  n={env.n} D={env.mpo_bond_dim} flops/apply={env.flops_per_apply:.3e}")
    x = env.pack(M.random_two_site_vector(mps, 5))
    z = env.pack(M.random_two_site_vector(mps, 6))
    ax = _apply(torch, env, x, "fp64")
    az = _apply(torch, env, z, "fp64")
    lhs, rhs = float(z @ ax), float(az @ x)
    scale = np.linalg.norm(ax) * np.linalg.norm(z)
    say(f"  <z,Ax>={lhs:.15e} <Az,x>={rhs:.15e}")
    assert abs(lhs - rhs) <= 1e-12 * scale
    ax32 = _apply(torch, env, x, "fp32")
    axbf = _apply(torch, env, x, "bf16x3")
    say(f"  fp32 vs fp64 {rel(ax32, ax):.3e}  bf16x3 vs fp64 {rel(axbf, ax):.3e}")
    assert rel(ax32, ax) <= 1e-5
    assert rel(axbf, ax) <= 1e-4
    # determinism: a second FP64 application is bitwise identical
    ax2 = _apply(torch, env, x, "fp64")
    assert np.array_equal(ax, ax2)
    # the plan the benchmark times (the shipped tuning cache: column-major intermediate,
    # channel-major phase 2, tuned tile costs and split-K, per-launch kernel choice) gives the
    # same product: FP64 to rounding, FP32 within the FP32 tolerance
    import os
    from paper_1509_00216_amd import lcc as L
    tctx = L.Context(0)
    tctx.set_tune_cache(os.path.join(os.path.dirname(L.LIB_PATH), "tune_cache.txt"))
    tenv = tctx.build_environments(tctx.create_hamiltonian(spec), mps)
    prof = tenv.profile_launches(to_dev(torch, x, torch.float32), to_dev(torch, x, torch.float32), "fp32", reps=1)
    say(f"  tuned plan: {len(prof)} launches, A k-major in {sum(p['a_kmajor'] for p in prof if p['kind'] == 'gemm')}")
    tx = _apply(torch, tenv, x, "fp64")
    tx32 = _apply(torch, tenv, x, "fp32")
    say(f"  tuned vs default plan: fp64 {rel(tx, ax):.3e}  fp32 {rel(tx32, ax):.3e}")
    assert rel(tx, ax) <= 1e-12
    assert rel(tx32, ax) <= 1e-5
