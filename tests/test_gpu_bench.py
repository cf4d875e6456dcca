"""bench.py end to end on the GPU at a reduced step count: one JSON line with
the fields of the benchmark contract, a roofline for the FP64 bounds kernel
on the default 2M-triangle workload, and the mixed forms against their own
four-slot VALU ceiling.  (The CPU oracle, second workload, backward and
variant legs are skipped here; the full run times them.)"""

import json
import os
import subprocess
import sys

import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_json_line():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    cmd = [sys.executable, "-u", os.path.join(ROOT, "bench.py"), "--steps", "2", "--warmup", "1",
           "--no-cpu-baseline", "--no-backward", "--no-variants", "--no-3d", "--no-second",
           "--no-fr"]
    print("[bench-test]", " ".join(cmd[2:]), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [ln for ln in r.stdout.splitlines() if ln.strip()]
    assert len(lines) == 1, r.stdout
    d = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
              "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config", "roofline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == 2 and d["warmup"] == 1
    assert d["value"] > 0 and d["ms_per_step"] > 0 and d["higher_is_better"] is True
    assert d["dtype"] == "f64" and d["data"] == "synthetic" and d["vs_baseline"] is None
    assert d["config"]["workload"].startswith("tri2m")
    assert d["config"]["stencil_elements"]["min"] >= 11
    roof = d["roofline"]
    assert roof["bound"] == "alu" and roof["unit"] == "TOP/s"
    assert 0.0 < roof["frac"] <= 1.0
    assert abs(roof["frac"] - roof["achieved"] / roof["peak"]) < 1e-9
    assert roof["traffic"] is None or roof["traffic"] > 0
    for name in ("fp32_valu", "fp16_mfma", "bf16_mfma"):
        m = d["mixed"][name]
        assert m["roofline"]["ops_per_pair"] == 4
        assert 0.0 < m["roofline"]["frac"] <= 1.0
        assert abs(m["roofline"]["frac"] - m["roofline"]["achieved"] / m["roofline"]["peak"]) < 1e-9
        if name != "fp32_valu":
            assert 0.0 < m["mfma"]["frac"] < 1.0
    print(f"[bench-test] value {d['value']:.4g} {d['unit']}, frac {roof['frac']:.3f}, "
          f"traffic {roof['traffic']}", flush=True)
