"""bench.py's host logic without a GPU: the refusal of several GPUs, the
algorithmic byte model of a sweep launch (per (source, rhs) the input and
output rows once, per source the packed state once, the block matrices once),
and the rule that the committed fabric-traffic figure is reported only while
the kernel sources it was measured on are unchanged."""
import json
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_several_gpus_are_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


def test_algorithmic_bytes_of_a_small_state():
    # 10 nodes, 27 couplings, one dense 3-node block and one 20-coupling
    # iterative block, 16 rhs in FP64: inputs and outputs 2*8*10*16 = 2560
    # bytes, couplings 27*(8+4) = 324, diagonal scale and indices 10*(4+8+4)
    # = 160, dense block 8*9 = 72, iterative block 12*20 = 240
    st = {"N": 10, "E": 27, "sum_k2": 9 + 400, "dense_k2": 9, "iter_nnz": 20}
    assert bench.algorithmic_bytes([st], 16, 8, 8) == 2560 + 324 + 160 + 72 + 240
    # two sources: twice the bytes; FP32 values and weights halve the rows and weights
    assert bench.algorithmic_bytes([st, st], 16, 8, 8) == 2 * (2560 + 324 + 160 + 72 + 240)
    assert bench.algorithmic_bytes([st], 16, 4, 4) == 1280 + 27 * 8 + 10 * 12 + 72 + 240


def test_layout_bytes_count_the_broadcast_input_once():
    st = {"N": 10, "E": 27, "sum_k2": 9}
    per = 2 * 8 * 10 * 16 + (8 + 32) * 10 + 72
    assert bench.layout_bytes([st, st], 16, 8, 8) == 2 * per
    assert bench.layout_bytes([st, st], 16, 8, 8, broadcast_once=True) == 2 * per - 8 * 10 * 16


def test_traffic_figure_follows_the_kernel_sources(tmp_path, monkeypatch):
    prof = os.path.join(ROOT, "profiles", "traffic_k_split_c4_fp64.json")
    if not os.path.exists(prof):
        pytest.skip("no committed traffic profile")
    # a copy of the tree's kernel sources and the profile under a scratch root
    for src in bench.KERNEL_SOURCES:
        os.makedirs(tmp_path / os.path.dirname(src), exist_ok=True)
        shutil.copy(os.path.join(ROOT, src), tmp_path / src)
    os.makedirs(tmp_path / "profiles")
    shutil.copy(prof, tmp_path / "profiles")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    with open(prof) as f:
        doc = json.load(f)
    got = bench.measured_traffic("k_split", "c4", "fp64")
    # the committed figure when the sources hash as recorded, else nothing
    import hashlib
    h = hashlib.sha256()
    for src in doc["kernel_sources"]:
        with open(os.path.join(ROOT, src), "rb") as f:
            h.update(f.read())
    expect = doc["per_launch"]["J"]["hbm_bytes"] if h.hexdigest() == doc["kernel_source_sha256"] else None
    assert got == expect
    with open(tmp_path / bench.KERNEL_SOURCES[0], "a") as f:
        f.write("\n// changed\n")
    assert bench.measured_traffic("k_split", "c4", "fp64") is None
    assert bench.measured_traffic("k_split", "c9", "fp64") is None
