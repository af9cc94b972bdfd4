"""Host logic of bench.py (no GPU): the multi-GPU refusal, the algorithmic
byte count of one sweep step, and the oracle baseline's bounded sample."""
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_1507_06565_amd import workloads as W  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_algorithmic_bytes():
    # 19 loads + 19 stores of FP32 per fluid cell, a 4 B word per cell, 12 B per link
    assert bench.algorithmic_bytes(1, 0, 0) == 152
    assert bench.algorithmic_bytes(0, 1, 0) == 4
    assert bench.algorithmic_bytes(0, 0, 1) == 12
    assert bench.algorithmic_bytes(97_177_700, 134_217_728, 48_735_228) == 15_892_704_048


def test_cpu_baseline_bounded_sample():
    import oracle
    rng = np.random.default_rng(3)
    S = W.quantise(np.column_stack([rng.uniform(0, 24, 6), rng.uniform(0, 16, 6), rng.uniform(2, 20, 6),
                                    rng.uniform(2.5, 5.0, 6)]))
    d = W.Domain(24, 16, 24, spheres=S, bc="cli")
    p = W.Params(collision="trt", tau_plus=0.7, magic_lambda=3 / 16, force=(5e-7, 0, 0))
    fl = oracle.flags(d)
    geo = (fl,) + oracle.links(d, fl)
    r = bench.cpu_baseline(d, p, geo, 4, 8, budget_s=0.5)
    assert r["kind"] == "oracle" and r["unit"] == "MLUPS" and r["value"] > 0 and r["cores"] >= 1
    assert "24x16x8 slab (z 4..11)" in r["sample"]
