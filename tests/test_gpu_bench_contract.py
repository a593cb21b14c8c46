"""bench.py's one JSON line, on a short run (the central Pb-Pb collision, the
tracker with the refit and merge legs, the oracle on one unit): every field
the line promises is there, with sane values, and the roofline objects
(the dominant kernel's, the refit's, the chain fit's) price what they say."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _roofline_ok(r):
    assert r["bound"] in ("hbm", "mfma", "alu")
    assert r["unit"] in ("GB/s", "TFLOP/s")
    assert r["achieved"] > 0 and r["peak"] > 0
    assert abs(r["frac"] - r["achieved"] / r["peak"]) <= 1e-9 * r["frac"]
    assert 0 < r["frac"] < 1
    assert "traffic" in r


def test_bench_line_keeps_its_contract():
    cmd = [sys.executable, "-u", "bench.py", "--workload", "pbpb_central", "--steps", "3", "--warmup", "1",
           "--cpu-units", "1", "--no-serve", "--no-batched", "--no-plain", "--no-collisions", "--no-clusterizer",
           "--no-compression"]
    print("case bench contract:", " ".join(cmd[1:]), flush=True)
    p = subprocess.run(cmd, cwd=ROOT, capture_output=True, text=True, timeout=280)
    assert p.returncode == 0, p.stderr[-2000:]
    lines = [ln for ln in p.stdout.splitlines() if ln.strip()]
    js = [ln for ln in lines if ln.lstrip().startswith("{")]
    assert len(js) == 1 and lines[-1] == js[0], lines[-3:]  # one JSON line, the last; the log goes to stderr
    d = json.loads(js[0])
    assert d["metric"] and d["unit"] == "clusters/s" and d["value"] > 0
    assert d["n_gpus"] == 1 and d["steps"] == 3 and d["warmup"] == 1
    assert d["higher_is_better"] is True and d["scaling"] in ("weak", "strong")
    assert d["vs_baseline"] is None and d["data"] == "synthetic" and d["dtype"]
    assert d["config"]["workload"] == "pbpb_central" and d["config"]["units"] == 36
    # value is the whole job's throughput over the timed steps
    assert abs(d["value"] * d["ms_per_step"] * 1e-3 - d["config"]["clusters"]) <= 1e-6 * d["config"]["clusters"]
    _roofline_ok(d["roofline"])
    assert d["roofline"]["kernel"] in d["kernel_ms"]
    c = d["cpu_baseline"]
    assert c["kind"] == "oracle" and c["value"] > 0 and c["cores"] >= 1 and c["unit"] and c["sample"]
    _roofline_ok(d["refit"]["roofline"])
    _roofline_ok(d["merge"]["chain_fit"]["roofline"])
    assert d["merge"]["links"] > 0 and d["refit"]["refitted_fraction"] > 0.98
