"""Host logic of bench.py that the committed profiles depend on: naming the timed kernel from a
launch profile (operand layouts, tile shape, kernel variant) and looking up its HBM traffic per
launch size (no GPU)."""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _launch(**kw):
    base = {"phase": 2, "kind": "gemm", "tile": (128, 64), "packed": False, "a_kmajor": True, "b_colmajor": True}
    base.update(kw)
    return base


def test_kernel_name_follows_layouts_and_variant():
    assert bench.kernel_name("fp32", _launch()) == "gemm_terms_kernel<1, true, true, 128, 64, 2, 2>"
    assert bench.kernel_name("fp64", _launch(a_kmajor=False)) == "gemm_terms_kernel<0, false, true, 128, 64, 2, 2>"
    assert bench.kernel_name("fp32", _launch(tile=(16, 64), packed=True, b_colmajor=False)) == \
        "gemm_packed_kernel<1, true, false, 16, 64, 1, 4>"
    assert bench.kernel_name("bf16x3", _launch(tile=(64, 16))) == "gemm_bf16x3_terms_kernel<true, true, 64, 16, 4, 1>"
    assert bench.kernel_name("fp32", {"kind": "reduce"}) == "reduce_kernel<float>"
    # 128x128 tiles: eight waves of 32x64 in FP32/FP64, four waves of 64x64 in BF16x3
    assert bench.kernel_name("fp32", _launch(tile=(128, 128), a_kmajor=False)) == \
        "gemm_terms_kernel<1, false, true, 128, 128, 4, 2>"
    assert bench.kernel_name("bf16x3", _launch(tile=(128, 128), a_kmajor=False)) == \
        "gemm_bf16x3_terms_kernel<false, true, 128, 128, 2, 2>"


def test_traffic_lookup_is_per_launch_size_and_source_digest():
    path = os.path.join(ROOT, "profiles", "pmc_traffic_abinitio_k24_m1000.txt")
    rec = json.load(open(path))
    key = max(rec["kernels"], key=lambda k: rec["kernels"][k]["traffic_bytes"])
    name, tiles = key.rsplit(" x", 1)
    got = bench.measured_traffic(name, int(tiles), "abinitio_k24_m1000")
    if rec["source_sha1"] == bench.source_digest():
        assert got == rec["kernels"][key]["traffic_bytes"]
        assert bench.measured_traffic(name, int(tiles) + 1, "abinitio_k24_m1000") is None
    else:  # counters taken on other kernel sources are not reported
        assert got is None
    assert bench.measured_traffic(name, int(tiles), "no_such_workload") is None


def test_more_than_one_gpu_is_refused():
    import subprocess
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
