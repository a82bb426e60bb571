"""Host logic of bench.py: the one-GPU contract and the HBM-traffic bookkeeping (counter
collections scaled by a calibration copy, invalidated when the kernel source changes)."""
import argparse
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


def _csv(path, counter, rows):
    with open(path, "w") as f:
        f.write("Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value\n")
        for d, name, v in rows:
            f.write(f'{d},"{name}",{counter},{v}\n')


def test_traffic_from_counter_collections(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_hash", lambda paths: "h1")
    (tmp_path / "profiles").mkdir()
    kib = bench.CALIB_BYTES / 1024
    das = "void usbf::das_tile_kernel<true, 4, 32, 4, false>(short const*)"
    fetch, write = tmp_path / "f.csv", tmp_path / "w.csv"
    # two counter rows per dispatch (summed); the copy reads half its bytes on this counter
    _csv(fetch, "FETCH_SIZE", [(1, das, 600.0), (1, das, 400.0), (2, das, 1000.0), (3, "elementwise_kernel", kib / 4),
                               (3, "elementwise_kernel", kib / 4)])
    _csv(write, "WRITE_SIZE", [(1, das, 64.0), (2, das, 64.0), (3, "elementwise_kernel", kib)])
    bench.write_traffic(argparse.Namespace(traffic_from=[str(fetch), str(write)], frames=0, traffic_command="cmd"))
    d = json.load(open(tmp_path / "profiles" / "traffic.json"))["das"]
    assert d["counters"]["FETCH_SIZE"]["scale"] == 2.0 and d["counters"]["WRITE_SIZE"]["scale"] == 1.0
    assert d["counters"]["FETCH_SIZE"]["launches"] == 2
    assert d["bytes_per_launch"] == 1000 * 1024 * 2.0 + 64 * 1024
    assert bench.traffic_from_profile("das", 32) == d["bytes_per_launch"]
    assert bench.traffic_from_profile("das", 16) is None          # another batch size
    monkeypatch.setattr(bench, "kernel_hash", lambda paths: "h2")
    assert bench.traffic_from_profile("das", 32) is None          # the kernel source changed


def test_kernel_hash_ignores_comments_only():
    a = 'int f(int x) { // the sum\n  return x + 1; /* one */ }\nconst char* s = "a // b";'
    b = 'int f(int x) {\n\n  return x + 1;   }   const char* s = "a // b";'
    c = 'int f(int x) { return x + 2; } const char* s = "a // b";'
    d = 'int f(int x) { return x + 1; } const char* s = "a  b";'
    assert bench.code_tokens(a) == bench.code_tokens(b)
    assert bench.code_tokens(a) != bench.code_tokens(c)   # a changed constant
    assert bench.code_tokens(a) != bench.code_tokens(d)   # a changed string literal


def test_committed_traffic_matches_the_current_kernel():
    """profiles/traffic.json describes the delay-and-sum source as it is in the tree."""
    assert bench.traffic_from_profile("das", 32) is not None


def test_beams_excludes_unused_line_slots():
    import synth
    assert bench.beams(synth.config_overlap_2d()) == 128 + 2 * 127
    assert bench.beams(synth.config_multiline_2d()) == 256
