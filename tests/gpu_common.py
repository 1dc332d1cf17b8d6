"""Shared helpers of the GPU tests (marshalling only; no arithmetic of the method)."""
import sys

import numpy as np
import pytest


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def need_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1509_00216_amd import lcc
    lcc.library()  # raises if the HIP library is missing: no fallback
    return torch, lcc


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def to_dev(torch, arr, dtype):
    return torch.tensor(np.asarray(arr), dtype=dtype, device="cuda:0").contiguous()


def product_mpo(ham):
    """The library's MPO in the oracle's dict format (input to the oracle's flop count only):
    channel shifts per bond and {(w_in, w_out): 4x4} per site, read through the C ABI."""
    K = ham.n_orb
    dq = []
    for b in range(K + 1):
        dn, dz = ham.channels(b)
        dq.append([(int(a), int(c)) for a, c in zip(dn, dz)])
    W = []
    for j in range(K):
        wi, wo, m = ham.site_mpo(j)
        W.append({(int(a), int(b)): mm for a, b, mm in zip(wi, wo, m)})
    return {"dq": dq, "W": W, "n_sites": K}
