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


def _counter_csv(path, counter, rows):
    cols = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id",
            "Grid_Size", "Kernel_Id", "Kernel_Name", "Workgroup_Size", "Counter_Name",
            "Counter_Value"]
    with open(path, "w") as fh:
        fh.write(",".join(f'"{c}"' for c in cols) + "\n")
        for i, (name, grid, value) in enumerate(rows, 1):
            fh.write(f'{i},{i},"Agent 1",1,1,1,{grid},7,"{name}",256,"{counter}",{value}\n')


def test_write_traffic_from_counter_csvs(tmp_path, monkeypatch):
    """The traffic entry comes from the two counter runs: the copy calibrates
    FETCH_SIZE (reads = writes), the last FP64 bounds launch is the profiled
    one (autotuner candidates at the same grid come earlier), and an entry of
    the same workload, kernel and grid is replaced, others kept."""
    (tmp_path / "profiles").mkdir()
    tf = tmp_path / bench.TRAFFIC_FILE
    tf.write_text("# header\n\n[entry]\nworkload = other\nkernel = k\ngrid_threads = 1\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_sources_sha", lambda dim: "ab" * 32)
    k_cand = "void kbl::(anonymous namespace)::bounds_fp64_1d<64, 1>(kbl::BoundsArgs)"
    k_main = "void kbl::(anonymous namespace)::bounds_fp64_1d<256, 1>(kbl::BoundsArgs)"
    copy = "__amd_rocclr_copyBuffer"
    _counter_csv(tmp_path / "f.csv", "FETCH_SIZE",
                 [(copy, 1024, 500.0), (k_cand, 64 * 64, 9.0), (k_main, 64 * 256, 30.0),
                  (k_main, 64 * 256, 34.0)])
    _counter_csv(tmp_path / "w.csv", "WRITE_SIZE",
                 [(copy, 1024, 1000.0), (k_cand, 64 * 64, 1.0), (k_main, 64 * 256, 3.0),
                  (k_main, 64 * 256, 5.0)])
    for _ in range(2):                                   # the second call replaces the entry
        e = bench.write_traffic("line64", str(tmp_path / "f.csv"), str(tmp_path / "w.csv"))
    assert e["kernel"] == "bounds_fp64_1d<256, 1>" and e["grid_threads"] == str(64 * 256)
    assert float(e["fetch_scale"]) == pytest.approx(2.0)
    assert float(e["bytes_per_launch"]) == pytest.approx((32.0 * 2.0 + 4.0) * 1024.0)
    # line64: 64 elements x 4 nodes x 3 variables read, rowptr, 3-element rows, bounds, status
    assert int(e["algorithmic_bytes_per_launch"]) == 64 * 4 * 3 * 8 + 65 * 4 + 192 * 4 + 6 * 64 * 8 + 64 * 4
    text = tf.read_text()
    assert text.count("[entry]") == 2 and "workload = other" in text
    assert text.startswith("# header")
