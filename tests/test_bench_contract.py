"""Host-side checks of the benchmark script's contract (no GPU): one GPU
only, and every HBM traffic figure it reports backed by a committed
counter summary."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT,
                       capture_output=True, text=True, timeout=300)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def _forms(v):
    """Ways a byte count is written in the summaries (MB or GB)."""
    mb, gb = v / 1e6, v / 1e9
    return {f"{mb:.2f}", f"{mb:.1f}", f"{gb:.1f}", f"{gb:.2f}"}


def test_traffic_figures_come_from_counter_summaries():
    sys.path.insert(0, ROOT)
    import bench

    text = ""
    pdir = os.path.join(ROOT, "profiles")
    for name in sorted(os.listdir(pdir)):
        with open(os.path.join(pdir, name), encoding="utf-8") as f:
            text += f.read()
    assert "--pmc FETCH_SIZE" in text and "--pmc WRITE_SIZE" in text
    missing = [key for key, v in bench.TRAFFIC.items() if not any(s in text for s in _forms(v))]
    assert not missing, missing
