"""Host-side parts of the benchmark: the single-GPU guard and the projection
fit report (host float64 library fits against the oracle's) at a small size."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "exactly one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


def test_fit_report_small():
    sys.path.insert(0, ROOT)
    import bench
    import paper_2312_16335_amd as lv
    from synth import gen

    lv.load()
    wl = gen.WORKLOADS["ood-1m-512"].scaled(m_learn=2000)
    r = bench.fit_report(lv, wl, n_s=3000, m_test=40)
    fits = r["fits"]
    assert set(fits) == {"id", "es", "fw", "fw_from_zero", "es_then_fw"}
    assert fits["id"]["max_abs_diff_vs_oracle"] < 1e-9
    assert abs(fits["es"]["beta"] - fits["es"]["beta_oracle"]) < 1e-6
    for name in ("es", "fw", "fw_from_zero", "es_then_fw"):
        f = fits[name]
        assert abs(f["loss"] - f["loss_oracle"]) <= 1e-6 * abs(f["loss_oracle"]), name
        assert 0.0 <= f["recall"] <= 1.0
    for name in ("fw", "fw_from_zero", "es_then_fw"):
        assert fits[name]["iters"] == fits[name]["iters_oracle"], name
    assert r["second_moments"]["max_rel_diff"] < 1e-12
    assert np.isfinite([f["lib_s"] for f in fits.values()]).all()
