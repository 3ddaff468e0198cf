"""bench.py end to end on a small workload (the 101 x 101 x 51 grid, 8
sources x 16 rhs): one JSON line on stdout with the fields its contract
names, the roofline fraction equal to achieved / peak, the node split's
placement report, the CPU-oracle baseline on one source, and the sweeping
baseline agreeing with the SCC/BTF output."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

pytestmark = [pytest.mark.gpu, pytest.mark.slow, pytest.mark.timeout(600)]


def test_bench_json_line_on_a_small_workload():
    print("case bench.py --config c3 --steps 3 --warmup 1", flush=True)
    r = subprocess.run([sys.executable, "-u", os.path.join(ROOT, "bench.py"), "--config", "c3", "--steps", "3",
                        "--warmup", "1", "--cpu-sources", "1", "--roofline-reps", "3"],
                       capture_output=True, text=True, timeout=540)
    assert r.returncode == 0, r.stderr[-3000:]
    lines = [ln for ln in r.stdout.strip().splitlines() if ln.strip()]
    assert len(lines) == 1, r.stdout
    d = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
              "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == 3 and d["warmup"] == 1 and d["dtype"] == "f64"
    assert d["value"] > 0 and d["ms_per_step"] > 0 and d["higher_is_better"] is True
    assert d["config"]["sources"] == 8 and d["config"]["rhs"] == 16
    # value = paired applies (sources x rhs) per second of the timed steps
    assert abs(d["value"] - 8 * 16 / (d["ms_per_step"] * 1e-3)) <= 1e-3 * d["value"]
    roof = d["roofline"]
    assert roof["bound"] == "hbm" and roof["unit"] == "GB/s" and roof["peak"] == 8000.0
    assert abs(roof["frac"] - roof["achieved"] / roof["peak"]) <= 1e-3
    assert abs(roof["achieved"] - roof["bytes_per_launch"] / (roof["launch_ms"] * 1e-3) / 1e9) <= 1e-3 * roof["achieved"]
    if d["config"]["schedule"]["split"] > 1:
        assert roof["placement"]["sources"] == 8
    cpu = d["cpu_baseline"]
    assert cpu["kind"] == "oracle" and cpu["value"] > 0 and cpu["cores"] >= 1
    sw = d["sweeping_baseline"]
    assert sw["agrees"] and sw["rel_l2_vs_scc_btf_J"] <= sw["agreement_tol"]
    print(f"  value {d['value']:.1f} {d['unit']}, frac {roof['frac']}, vs sweeping {d['vs_sweeping']}", flush=True)
