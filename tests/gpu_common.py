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
