"""Host logic of bench.py (no GPU): the one-GPU guard, the counter-file
traffic arithmetic (calibration scaling), and the algorithmic-byte count."""
import csv
import json
import os
import subprocess
import sys

import numpy as np

import bench
from paper_2607_18541_amd import lz

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def _counter_csv(path, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Counter_Value"])
        w.writeheader()
        for name, kib in rows:
            w.writerow({"Kernel_Name": name, "Counter_Value": kib})


def test_traffic_scaled_by_the_calibration_kernel(tmp_path, monkeypatch):
    # the calibration kernel reads and writes n bytes; this FETCH counter
    # reports half of them and WRITE all of them, so fetch is scaled by 2
    n = 1 << 20
    parse = "void (anonymous namespace)::k_lz<64, 2, 3, false>((anonymous namespace)::KArgs)"
    depth = "void (anonymous namespace)::k_lz<64, 2, 1, false>((anonymous namespace)::KArgs)"
    cal = "void at::native::vectorized_elementwise_kernel<16, bitwise_not_kernel_cuda>"
    steps = 2
    _counter_csv(tmp_path / "f.csv", [(parse, 100), (parse, 100), (depth, 10), (depth, 10), (depth, 10),
                                      (depth, 10), (cal, n / 2 / 1024)])
    _counter_csv(tmp_path / "w.csv", [(parse, 300), (parse, 300), (depth, 5), (depth, 5), (depth, 5),
                                      (depth, 5), (cal, n / 1024)])
    monkeypatch.setattr(bench, "TRAFFIC_JSON", str(tmp_path / "t.json"))
    out = bench.traffic_from_counters(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), steps, n, "cmd")
    assert out["fetch_scale"] == 2.0 and out["write_scale"] == 1.0
    p = out["kernels"]["k_lz<64, 2, 3, false>"]
    assert p["launches_per_decode"] == 1.0
    assert p["fetch_bytes_per_decode"] == 100 * 1024 * 2
    assert p["write_bytes_per_decode"] == 300 * 1024
    d = out["kernels"]["k_lz<64, 2, 1, false>"]
    assert d["launches_per_decode"] == 2.0
    assert d["traffic_bytes_per_decode"] == 2 * (10 * 1024 * 2 + 5 * 1024)
    assert "calibration" not in out["kernels"]
    assert json.load(open(tmp_path / "t.json"))["source_sha256"] == bench.source_digest()


def test_algorithmic_bytes_of_a_hand_built_archive():
    # one block of 40 bytes: literals "abcd", a 12-byte match, 4 literals, the
    # block's last token ends with a 20-byte implied match
    lit = np.frombuffer(b"abcdwxyz", np.uint8)
    ll, ml, sr = [4, 4], [12, 20], [0, 3]
    n = 40
    arc = lz.build_archive(n, 12, ll, ml, sr, lit)
    info = lz.archive_info(arc)
    assert info["match_bytes"] == 32 and info["n_blocks"] == 1
    alg, tok = bench.algorithmic_bytes(arc, info)
    c = bench.header_counts(arc)
    assert c["n_tok"] == 2 and c["n_lit"] == 8
    # tokens: 1 cmd byte + 4 source bytes each, the extension words, the block table
    assert tok == 2 * 5 + 2 * c["n_x16"] + 4 * c["n_x32"] + 32 * 2
    # every output byte written once, every match and literal byte read once
    assert alg == 40 + 32 + 8 + tok
