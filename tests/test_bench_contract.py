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


def test_tape_window_decoding():
    """The adjoint-window split the bench prices the adjoint with, decoded
    from a tape laid out as include/cm.h documents: a pair recorded as
    indices, one as a bit mask and one not recorded."""
    import numpy as np
    import torch
    from types import SimpleNamespace
    K, cap = 8, 4
    stride = 16 + 80 * K
    hdr = (cap * stride + 255) // 256 * 256
    nvA = np.array([10, 6, 5])
    nvB = np.array([8, 4, 5])
    lists = [np.array([1, 9, 10, 17, 18, 40, 41]), None, None]        # pair 0: 2 of A, 2 of B, 3 E-E
    ncand1 = 6 + 4 + 2 * 20
    bits1 = np.zeros(64 * ((ncand1 + 63) // 64), np.uint8)
    bits1[[0, 5, 6, 9, 10, 11, 12, 30, 31]] = 1                         # pair 1: 2 of A, 2 of B, 5 E-E
    mask_words = np.packbits(bits1, bitorder="little").view(np.uint64)
    pool = np.zeros(64, np.int32)
    pool[0:7] = lists[0]
    pool[8:8 + 2 * len(mask_words)] = mask_words.view(np.int32)
    buf = np.zeros(256 + hdr + 4 * pool.size, np.uint8)
    buf[0:8] = np.array([8 + 2 * len(mask_words)], np.uint64).view(np.uint8)
    for p, (cnt, form, off) in enumerate(((7, 1, 0), (9, 2, 8), (5, 0, 0))):
        rec = 256 + p * stride
        buf[rec:rec + 8] = np.array([cnt, form], np.int32).view(np.uint8)
        buf[rec + 8:rec + 16] = np.array([off], np.int64).view(np.uint8)
    buf[256 + hdr:] = pool.view(np.uint8)
    out = SimpleNamespace(K=K, capacity=cap, n_pairs=torch.tensor([3], dtype=torch.int32),
                          tape=torch.from_numpy(buf))
    w_a, w_b, w_e = bench.tape_windows(out, nvA, nvB)
    assert w_a.tolist() == [2, 2, 0]
    assert w_b.tolist() == [2, 2, 0]
    assert w_e.tolist() == [3, 5, 5]
