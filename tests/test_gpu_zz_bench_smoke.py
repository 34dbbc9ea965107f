"""The benchmark runs end to end on the GPU (headline leg only, few steps) in a
child process and prints one JSON line with the fields of its contract."""
import json
import subprocess
import sys
from pathlib import Path

import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

ROOT = Path(__file__).resolve().parents[1]


def test_bench_prints_its_json_line():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print("bench smoke: headline leg, 2 steps", flush=True)
    r = subprocess.run([sys.executable, str(ROOT / "bench.py"), "--steps", "2", "--warmup", "1", "--no-cpu",
                        "--no-plain", "--no-grad", "--sweeps", "0", "--no-data", "--no-cov"],
                       capture_output=True, text=True, timeout=200, cwd=str(ROOT))
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [ln for ln in r.stdout.splitlines() if ln.strip()]
    assert len(lines) == 1
    d = json.loads(lines[0])
    for key in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
                "scaling", "vs_baseline", "dtype", "data", "config", "roofline"):
        assert key in d, key
    assert d["n_gpus"] == 1 and d["steps"] == 2 and d["warmup"] == 1
    assert d["value"] > 0 and d["ms_per_step"] > 0 and d["higher_is_better"] is True
    assert d["config"]["workload"] == "year_912085bins_4096states"
    rf = d["roofline"]
    assert rf["bound"] in ("alu", "hbm", "mfma") and 0 < rf["frac"] < 1 and rf["peak"] > 0
    assert rf["achieved"] == pytest.approx(rf["frac"] * rf["peak"], rel=1e-2)
    assert rf["traffic"] is not None and rf["traffic"] > 0
