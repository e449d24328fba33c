"""Host-side checks of bench.py: the roofline's traffic figure is read from
the committed counter summary only when that summary was taken on the
current kernel source, and more than one GPU is refused with a message."""
import os
import re
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _summary():
    kv = {}
    with open(os.path.join(ROOT, "profiles", "stream_kernel_4096_counters.md")) as fh:
        for line in fh:
            m = re.match(r"- (\S+): `([^`]*)`", line)
            if m:
                kv[m.group(1)] = m.group(2)
    return kv


def test_traffic_follows_the_kernel_source():
    kv = _summary()
    shapes = [k for k in kv if k.startswith("hbm_bytes_per_launch[")]
    assert shapes
    current = kv["kernel_sha"] == bench.kernel_sha()
    for k in shapes:
        c, t, r = (int(v) for v in k[k.index("[") + 1:-1].split(","))
        got = bench.read_traffic({"cols": c, "tsteps": t, "seg_rows": r}, 4096)
        # counters taken on another source are never reported
        assert got == (float(kv[k]) if current else None), k
    # a shape the summary does not list, and a size it does not cover
    assert bench.read_traffic({"cols": 1, "tsteps": 1, "seg_rows": 1}, 4096) is None
    assert bench.read_traffic({"cols": 2, "tsteps": 3, "seg_rows": 36}, 1234) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)
