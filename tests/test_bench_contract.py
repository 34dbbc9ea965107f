"""The benchmark's contract on the CPU: it refuses more than one GPU, and the
committed rocprofv3 summaries still describe the current kernel sources (so the
bench line carries their traffic and instruction figures instead of nulls)."""
import subprocess
import sys
from pathlib import Path

ROOT = Path(__file__).resolve().parents[1]
sys.path.insert(0, str(ROOT))

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, str(ROOT / "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_profiles_match_the_kernel_sources():
    w = "year_912085bins_4096states"
    # the launch shape the library picks for this batch by default (8 bins per
    # lane, six 21-state sub-tiles per work item)
    assert bench.profiled_traffic(w, (8, 126)) > 0
    assert bench.profiled_forward_field(w, "valu_lane_instr_per_state_bin_fp64") > 0
    assert bench.profiled_cov_valu() > 0
    assert bench.profiled_cov_grad_valu() > 0
