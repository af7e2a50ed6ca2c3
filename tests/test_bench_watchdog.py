"""bench.py host logic (no GPU): the leg watchdog (a leg that stops making
progress ends the run with one JSON line that keeps the results so far and
marks the stalled leg) and the one-GPU check."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r"""
import sys, time
sys.path.insert(0, %r)
import bench
bench.LEG_STALL_S = 1.0
result = {"metric": "m", "value": 1.5, "unit": "u", "serving": {"1e4": {"p50_us": 3}}}
current = [None]
bench.start_leg_watchdog(result, {"mandel": {"grid": 0}}, current)
time.sleep(2.5)              # no leg running: the watchdog stays quiet
bench.log("[test] progress")
current[0] = "serving"       # a leg that then stalls
time.sleep(30)
print("not reached")
"""


def test_stalled_leg_ends_the_run_with_one_json_line():
    p = subprocess.run([sys.executable, "-c", SCRIPT % ROOT], capture_output=True, text=True,
                       timeout=60)
    assert p.returncode == 0, p.stderr
    lines = [l for l in p.stdout.splitlines() if l.strip()]
    assert len(lines) == 1, p.stdout
    out = json.loads(lines[0])
    assert out["value"] == 1.5 and out["unit"] == "u"
    assert out["serving"]["1e4"] == {"p50_us": 3}       # what the leg measured is kept
    assert "no progress" in out["serving"]["error"]
    assert out["tuned"] == {"mandel": {"grid": 0}}
    assert "no progress" in p.stderr


def test_more_than_one_gpu_is_refused_with_a_message():
    """bench.py measures one GPU: any other --gpus value exits at once with a
    message (before touching a device)."""
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr and p.stdout == ""
