"""Pins of the oracle's full-size contraction (oracle.stacked): its channel-stacked environments
are the environments of oracle.blocksparse block for block, and its H_eff x equals the
Fock-space H_eff of O1, for both oracle MPOs (prefix automaton and two-sided labels)."""
import numpy as np
import pytest

from oracle import blocksparse as BS
from oracle import fock
from oracle import mpo as OM
from oracle import stacked as ST
from workloads import configs as C
from workloads import hamiltonians as H
from workloads import mps as M

CASES = {
    "chain8_complete": lambda: C.make("hubbard1d_k8_m64"),
    "abinitio_k6_m12": lambda: (H.random_ab_initio(6, 6, seed=21), M.random_mps(6, 6, 0, 12, seed=22)),
    "abinitio_k8_sz1_offcentre": lambda: (H.random_ab_initio(8, 5, two_sz=1, seed=3),
                                          M.random_mps(8, 5, 1, 30, seed=4, center=2)),
    "threeband_2x1_m10": lambda: (H.three_band(2, 1, n_holes=3, two_sz=1), M.random_mps(6, 3, 1, 10, seed=4)),
}


def _same_blocks(dict_env, stacked_blocks):
    for w, blocks in dict_env.items():
        for k, b in blocks.items():
            assert np.abs(stacked_blocks[w][k] - b).max() <= 1e-12 * max(1.0, np.abs(b).max())
    for w, blocks in stacked_blocks.items():  # anything else must be an untouched zero block
        for k, b in blocks.items():
            if w not in dict_env or k not in dict_env[w]:
                assert not np.any(b)


@pytest.mark.parametrize("builder", ["prefix", "twosided"])
@pytest.mark.parametrize("name", sorted(CASES))
def test_stacked_environments_and_apply(name, builder):
    spec, mps = CASES[name]()
    mpo = OM.build_mpo(spec) if builder == "prefix" else OM.build_mpo_twosided(spec)
    l = mps["center"]
    _same_blocks(BS.left_environments(mps, mpo, l),
                 ST.as_blocks(ST.left_environment(mps, mpo, l), mpo["dq"][l], mps["bonds"][l]))
    _same_blocks(BS.right_environments(mps, mpo, l + 2),
                 ST.as_blocks(ST.right_environment(mps, mpo, l + 2), mpo["dq"][l + 2], mps["bonds"][l + 2]))
    blocks = M.two_site_blocks(mps)
    x = M.random_two_site_vector(mps, 5)
    y1 = fock.effective_hamiltonian(spec, mps, blocks) @ BS.flatten(x, blocks)
    y = BS.flatten(ST.FullSizeEnvironments(spec, mps, mpo).apply(x), blocks)
    assert np.linalg.norm(y - y1) <= 1e-13 * np.linalg.norm(y1)
