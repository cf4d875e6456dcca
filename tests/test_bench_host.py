"""Host-side parts of bench.py: the traffic lookup in the committed counter
summary and the refusal of several GPUs.  No GPU is touched."""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _entries():
    out, cur = [], None
    for line in open(os.path.join(ROOT, bench.TRAFFIC_FILE)):
        line = line.strip()
        if line == "[entry]":
            cur = {}
            out.append(cur)
        elif "=" in line and cur is not None and not line.startswith("#"):
            k, v = line.split("=", 1)
            cur[k.strip()] = v.strip()
    return out


def test_traffic_entries_are_well_formed():
    """Every entry names its kernel, grid, workload and sources, and reports
    at least the algorithmic bytes.  (An entry whose sources have changed
    since the counters only makes bench report null traffic.)"""
    entries = _entries()
    assert "tri2m" in {e["workload"] for e in entries}
    for e in entries:
        assert e["kernel"].startswith("bounds_fp64_")
        assert int(e["grid_threads"]) > 0 and len(e["source_sha256"]) == 64
        assert float(e["bytes_per_launch"]) >= float(e["algorithmic_bytes_per_launch"])


def test_traffic_lookup_prefers_the_exact_grid_then_falls_back():
    e = next(x for x in _entries() if x["workload"] == "tri2m")
    if e["source_sha256"] != bench.kernel_sources_sha(2):
        pytest.skip("the 2D kernel sources changed since its counters were taken")
    k, g = e["kernel"], int(e["grid_threads"])
    exact = bench.profiled_traffic(k, g, "tri2m", 2)
    assert exact == (float(e["bytes_per_launch"]), g)
    other = bench.profiled_traffic(k, 256 * 8 * 256, "tri2m", 2)   # a persistent grid
    assert other == exact
    assert bench.profiled_traffic(k, g, "no_such_workload", 2) == (None, None)
    assert bench.profiled_traffic("bounds_fp64_2d<1, 1, 1, 1, 0>", g, "tri2m", 2) == (None, None)
    assert bench.profiled_traffic(k, g, "tri2m", 1) == (None, None)


def test_pair_ops():
    assert bench.pair_ops(1) == 8
    assert bench.pair_ops(2) == 6
    assert bench.pair_ops(3) == 6
    assert bench.MIXED_PAIR_OPS == 4


def test_mfma_flops_count():
    """64x64 grid, tile (2 x tiles, 4 k-steps, 2 waves): per element 4 x tiles,
    4 envelopes, 4 k-steps, 3 (FP16) or 6 (BF16) 16x16x16 MFMAs."""
    import types
    from paper_2407_20966_amd import _lib
    kbl = types.SimpleNamespace(_lib=_lib, PREC_MIXED_FP16=_lib.PREC_MIXED_FP16)
    wl = types.SimpleNamespace(n_elem=10)
    assert bench.mfma_flops_issued(wl, _lib.PREC_MIXED_FP16, 5, kbl) == 10 * 4 * 4 * 4 * 3 * 8192
    assert bench.mfma_flops_issued(wl, _lib.PREC_MIXED_BF16, 5, kbl) == 10 * 4 * 4 * 4 * 6 * 8192


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
