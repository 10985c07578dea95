"""Host-side checks of the benchmark script's contract: it runs on exactly one
GPU, and a stored HBM-traffic figure is reported only for the kernel sources
it was measured on."""
import json
import os
import re
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]


def test_stored_traffic_needs_matching_sources(tmp_path):
    h = bench.source_hash(bench.FWD_SOURCES)
    good = tmp_path / "good.md"
    good.write_text(f"source_hash: {h}\ntraffic_bytes_per_launch: 1.5e9\n")
    assert bench.stored_traffic(str(good), bench.FWD_SOURCES) == 1.5e9
    stale = tmp_path / "stale.md"
    stale.write_text("source_hash: 0123456789abcdef\ntraffic_bytes_per_launch: 1.5e9\n")
    assert bench.stored_traffic(str(stale), bench.FWD_SOURCES) is None
    assert bench.stored_traffic(str(tmp_path / "absent.md"), bench.FWD_SOURCES) is None
    # a figure stored for one kernel's sources is void for another's
    assert bench.stored_traffic(str(good), bench.EE_SOURCES) is None


def test_committed_traffic_summaries_are_parsable():
    for path, key in ((bench.TRAFFIC_FILE, "traffic_bytes_per_launch"),
                      (bench.EE_TRAFFIC_FILE, "smooth_traffic_bytes_per_launch"),
                      (bench.EE_TRAFFIC_FILE, "hard_traffic_bytes_per_launch")):
        txt = open(path).read()
        assert re.search(r"source_hash:\s*[0-9a-f]{16}", txt), path
        m = re.search(key + r":\s*([0-9.eE+]+)", txt)
        assert m and float(m.group(1)) > 0, (path, key)
