"""Host-side checks of bench.py and of the committed bench lines (no GPU).

* `--gpus N` with N > 1 exits with status 2 and a message (one GPU only).
* The HBM traffic of the build kernel is reported only for a workload and
  build whose counters are committed (profiles/hbm_traffic_k_direct_fused_*),
  never for the seed construction or a workload without counters.
* Every committed bench line under profiles/ carries the command that made it
  and the keys of the bench line; the default line (cfg3) also the roofline,
  the per-stage CPU oracle baseline, its accuracy against the oracle's stored
  solution and the refined split-BF16 against plain FP64 comparison.
"""
import glob
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

KEYS = ["metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
        "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config"]


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_traffic_only_for_its_own_workload():
    import bench
    for w in ("cfg2", "cfg3"):
        v = bench.measured_traffic(w, "fp32")
        assert v is None or v > 0  # None once the kernel sources changed since the counters
        assert bench.measured_traffic(w, "fp32", seed=True) is None
        assert bench.measured_traffic(w, "bf16x3") is None
    assert bench.measured_traffic("cfg1", "fp32") is None


@pytest.mark.parametrize("path", sorted(glob.glob(os.path.join(ROOT, "profiles", "bench_*.json"))),
                         ids=os.path.basename)
def test_committed_bench_lines(path):
    d = json.load(open(path))
    assert d["command"].startswith("python bench.py")
    for k in KEYS:
        assert k in d, k
    assert d["n_gpus"] == 1 and d["value"] > 0 and "workload" in d["config"]
    if os.path.basename(path) == "bench_cfg3_fp32.json":  # the default line
        assert d["command"] == "python bench.py"
        r = d["roofline"]
        assert r["bound"] == "mfma" and r["unit"] == "TFLOP/s" and r["peak"] == 157.3
        assert abs(r["frac"] - r["achieved"] / r["peak"]) < 1e-3
        c = d["cpu_baseline"]
        assert c["kind"] == "oracle" and c["cores"] >= 1 and c["value"] > 0 and c["sample"]
        assert c["host_cpus"] >= 1 and c["cpu_model"]
        assert set(c["stage_s"]) == {"build", "projection", "block_eigh", "spectrum"}
        a = d["accuracy_vs_oracle"]
        assert a["meets_bars"] and a["lowest100_max_err_eV"] < 1e-5 and a["eps2_rel_err"] <= 1e-4
        f = d["precision_forms"]
        for form in ("refined_bf16x3", "plain_fp64"):
            assert f[form]["solves_within_0.1meV"] == f[form]["solves"]
        assert f["refined_bf16x3_over_plain_fp64_at_0.1meV"] > 1
