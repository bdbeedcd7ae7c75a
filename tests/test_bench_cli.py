"""bench.py's contract on the host (no GPU): one GPU only, the traffic figure
tied to the ray caster's sources (null once they change), and the paper's own
figures carried as context with their hardware."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert msg["n_gpus"] == 2 and "one GPU" in msg["error"]


def test_traffic_is_reported_only_for_the_measured_sources():
    t = bench.RAYCAST_TRAFFIC
    assert t["bytes"] == int(round((t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"]) * 1024))
    # the counted bytes, or None once the ray caster's sources differ from those measured
    assert bench.raycast_traffic() in (None, t["bytes"])


def test_paper_figures_are_context_with_hardware():
    f = bench.PAPER_FIGURES
    assert "context" in f["note"]
    for key in ("otsu_256_bins_ms", "its_256_bins_ms", "best_view_search_s"):
        vals = [v for k, v in f[key].items() if k != "mean"]
        assert len(vals) == 5 and abs(sum(vals) / 5 - f[key]["mean"]) < 0.01 * f[key]["mean"]
    assert "Core i7" in f["threshold_hardware"] and "not stated" in f["best_view_hardware"]
