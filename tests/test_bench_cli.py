"""bench.py's command-line contract on the CPU: more than one GPU is refused with a
message and a non-zero exit, before anything touches a device."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode != 0
    line = [ln for ln in r.stdout.splitlines() if ln.startswith("{")][-1]
    assert "one GPU" in json.loads(line)["error"]
