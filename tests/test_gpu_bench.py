"""The benchmark's output contract on the GPU: one JSON line carrying the
fields its consumers read (metric, value, roofline, CPU baseline), checked
on a shrunken workload (4 shots, 100 steps, B = 2) that runs in seconds."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("extra", [[], ["--separate"], ["--ckpt-every", "0"]],
                         ids=["fused", "separate", "history"])
def test_bench_line_fields(extra):
    print(f"case: bench.py {' '.join(extra)} on 921x301, 4 shots, nt=100, B=2, one step",
          flush=True)
    cmd = [sys.executable, "-u", os.path.join(ROOT, "bench.py"), "--shots", "4", "--nt", "100",
           "--batch", "2", "--steps", "1", "--warmup", "0", "--cpu-nt", "20", *extra]
    r = subprocess.run(cmd, cwd=ROOT, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-3000:]
    lines = [ln for ln in r.stdout.splitlines() if ln.startswith("{")]
    assert len(lines) == 1, r.stdout[-3000:]
    d = json.loads(lines[0])
    for key in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
                "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config",
                "roofline", "cpu_baseline"):
        assert key in d, key
    assert d["n_gpus"] == 1 and d["steps"] == 1 and d["warmup"] == 0
    assert d["unit"] == "Hv/s" and d["higher_is_better"] is True and d["vs_baseline"] is None
    assert d["value"] > 0 and d["ms_per_step"] > 0 and "workload" in d["config"]
    assert d["config"]["ckpt_every"] == (0 if "--ckpt-every" in extra else 50)
    ro = d["roofline"]
    for key in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert key in ro, key
    assert ro["bound"] == "hbm" and ro["unit"] == "GB/s" and ro["peak"] == 8000.0
    assert 0 < ro["frac"] < 1.5 and abs(ro["frac"] - ro["achieved"] / ro["peak"]) < 1e-9
    # the committed counter runs are of the default workload's launches only
    assert ro["traffic"] is None
    cb = d["cpu_baseline"]
    for key in ("value", "unit", "cores", "kind", "sample"):
        assert key in cb, key
    assert cb["kind"] == "oracle" and cb["value"] > 0 and 1 <= cb["cores"] <= 4


def test_bench_refuses_a_workspace_larger_than_free_memory():
    """History mode on the full 64-shot, 4000-step workload would keep
    357 GB of forward levels: the bench says so and exits with status 2
    before allocating the workspace."""
    print("case: bench.py --ckpt-every 0 on the full 921x301, 64-shot, 4000-step workload",
          flush=True)
    cmd = [sys.executable, "-u", os.path.join(ROOT, "bench.py"), "--ckpt-every", "0",
           "--steps", "1", "--warmup", "0", "--no-cpu-baseline"]
    r = subprocess.run(cmd, cwd=ROOT, capture_output=True, text=True, timeout=600)
    assert r.returncode == 2, r.stderr[-3000:]
    assert "GB of workspace" in r.stderr and "history mode" in r.stderr
