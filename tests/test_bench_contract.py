"""The committed bench line keeps the contract of `bench.py`'s JSON output (CPU only: reads the
record under profiles/, runs nothing on a GPU)."""
import json
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_committed_bench_line_fields():
    d = json.load(open(os.path.join(ROOT, "profiles", "bench_chainring1000_line.json")))
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
              "scaling", "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["value"] > 0 and d["ms_per_step"] > 0
    assert d["config"]["workload"] == "chainring1000"
    r = d["roofline"]
    assert r["bound"] in ("hbm", "mfma", "alu") and r["unit"] in ("GB/s", "TFLOP/s")
    assert abs(r["frac"] - r["achieved"] / r["peak"]) < 1e-9
    c = d["cpu_baseline"]
    assert c["kind"] == "oracle" and c["cores"] >= 1 and c["value"] > 0 and c["sample"]
    # value is the sigma block's algorithmic flops over its measured time
    assert abs(d["value"] - d["sigma_block_flops"] / (d["ms_per_step"] * 1e-3) / 1e12) < 1e-6 * d["value"]


def test_traffic_record_matches_its_algorithmic_bytes():
    t = json.load(open(os.path.join(ROOT, "profiles", "exchange_m_chainring1000_traffic.json")))
    assert t["bytes_per_launch"] == t["fetch_bytes_per_launch"] + t["write_bytes_per_launch"]
    assert t["bytes_per_launch"] >= t["algorithmic_bytes_per_launch"]
    assert 0.4 < t["copy_calibration"]["fetch_factor"] < 1.1 and 0.4 < t["copy_calibration"]["write_factor"] < 1.1
