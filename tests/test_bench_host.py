"""Host-side parts of bench.py: the one-GPU guard and the oracle baseline
leg (no GPU needed for either)."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_cpu_baseline_fields():
    sys.path.insert(0, ROOT)
    import bench
    cb = bench.cpu_baseline()
    assert cb["kind"] == "oracle" and cb["unit"] == "s"
    assert isinstance(cb["cores"], int) and 1 <= cb["cores"] <= (os.cpu_count() or 1)
    assert cb["value"] > 0 and "32^3" in cb["sample"] and "64^3" in cb["sample"]
    with open(bench.ORACLE_RECORD) as f:
        rec = json.load(f)
    # the record is a measurement of the oracle at 64^3 (one pole, 8 sources)
    assert rec["factor_s"] > 0 and rec["solve_s"] > 0 and rec["ratio_hex64_over_hex32"] > 1
    assert "Model name" in rec["host"]
    json.dumps(cb)
