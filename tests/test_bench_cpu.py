"""bench.py's command-line contract that needs no GPU: more than one GPU is
refused with a message (the benchmark measures one GPU), and the counter
profile it reports traffic from is well formed."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_counter_profile_is_consistent():
    d = json.load(open(os.path.join(ROOT, "profiles", "vbatched_f32_kernel_uneven65536_counters.json")))
    cal = d["copy_calibration"]
    hbm = (d["fetch_size_kib_per_dispatch"] * 1024 * cal["fetch_scale"]
           + d["write_size_kib_per_dispatch"] * 1024 * cal["write_scale"])
    assert abs(hbm - d["hbm_bytes_per_launch"]) <= 1e-3 * hbm
    assert abs(cal["fetch_size_kib"] * 1024 * cal["fetch_scale"] - cal["bytes"]) <= 1e-3 * cal["bytes"]
    assert 0.9 < d["traffic_over_algorithmic"] < 1.5


def test_traffic_hash_follows_the_kernel_sources(tmp_path, monkeypatch):
    """The stored traffic applies while the batched kernel's file and its
    local headers are unchanged: the hash covers exactly that include
    closure (a change to another device source leaves it alone)."""
    sys.path.insert(0, ROOT)
    import bench
    h0 = bench.source_hash()
    # a copy of the tree's device sources; edit one file at a time
    import shutil
    src = os.path.join(ROOT, "paper_2208_09822_amd", "csrc")
    fake = tmp_path / "paper_2208_09822_amd" / "csrc"
    shutil.copytree(src, fake, ignore=shutil.ignore_patterns("*.o"))
    shutil.copytree(os.path.join(ROOT, "include"), tmp_path / "include")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.source_hash() == h0
    with open(fake / "xgemm.hip", "a") as f:  # not included by the batched kernel
        f.write("\n// edit\n")
    assert bench.source_hash() == h0
    with open(fake / "tiles.h", "a") as f:  # included (through batched.hip)
        f.write("\n// edit\n")
    assert bench.source_hash() != h0
