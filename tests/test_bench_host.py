"""Host logic of bench.py: the JSON record's contract fields, the roofline
arithmetic and the single-GPU guard (no GPU needed)."""
import json
import os
import subprocess
import sys

import bench
from workloads import planted

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def fake_run():
    A = planted(300, 200, 150, 6, 1)
    info = {"s": 8, "len": 52, "check_terms": 4, "t_sequence": 0.01, "t_sigma": 0.02, "sigma_threads": 4}
    us = {65521: [10.0, 20.0, 0.0], 2**31 - 1: [12.0, 24.0, 0.0]}
    plan = {"W": 8, "G1": 2, "G2": 4, "fused": 1, "NB": 64, "esize": 2}
    return A, [info, info], us, {65521: plan, 2**31 - 1: dict(plan, esize=4)}


def test_result_line_contract():
    A, infos, us, plans = fake_run()
    out = bench.result_line(A, 8, (65521, 2**31 - 1), 1, 1, 0.5, infos, us, plans)
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
              "vs_baseline", "dtype", "data", "config", "roofline"):
        assert k in out, k
    assert out["config"]["workload"] and out["n_gpus"] == 1 and out["vs_baseline"] is None
    work = 2 * (2.0 * A.nnz * 8 * 55)
    assert abs(out["value"] - round(work / 0.5 / 1e9, 3)) < 1e-9
    rf = out["roofline"]
    b2 = 4 * (A.n + 1) + 5 * A.nnz + 4 * 8 * (A.m + A.n)
    assert rf["bytes_per_launch"] == b2
    assert abs(rf["achieved"] - round(b2 / 20e-6 / 1e9, 1)) < 1e-9
    assert abs(rf["frac"] - round(rf["achieved"] / 8000.0, 4)) < 1e-4
    json.dumps(out)


def test_traffic_is_null_without_matching_summary(tmp_path, monkeypatch):
    import hashlib

    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.kernel_traffic(8, 4, 2, True) is None
    (tmp_path / "profiles").mkdir()
    (tmp_path / "paper_0704_2351_amd" / "csrc").mkdir(parents=True)
    (tmp_path / "paper_0704_2351_amd" / "csrc" / "spmm.hip").write_text("kernel v2")
    name16 = "k_spmm_split<8, 4, 1, true, true, unsigned short, 0>"
    name32 = "k_spmm_split<8, 4, 2, false, true, unsigned int, 0>"
    rec = {"source": "paper_0704_2351_amd/csrc/spmm.hip", "source_sha256": "0" * 64,
           "kernels": {name16: {"bytes_per_launch": 123}, name32: {"bytes_per_launch": 456}}}
    (tmp_path / "profiles" / "traffic.json").write_text(json.dumps(rec))
    assert bench.kernel_traffic(8, 4, 2, True) is None  # another revision of the source
    rec["source_sha256"] = hashlib.sha256(b"kernel v2").hexdigest()
    (tmp_path / "profiles" / "traffic.json").write_text(json.dumps(rec))
    assert bench.kernel_traffic(8, 4, 2, True) == 123
    assert bench.kernel_traffic(8, 4, 4, True) == 456
    assert bench.kernel_traffic(8, 8, 2, True) is None  # instantiation not measured
    assert bench.kernel_traffic(8, 4, 2, False) is None


def test_committed_traffic_record_matches_source():
    """The committed counter summary belongs to the current kernel source and holds the instantiations
    the autotuner picks on the 200000 x 150000 workload at p = 65521."""
    rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    assert bench.kernel_traffic(8, 4, 2, True) == rec["kernels"][
        "k_spmm_split<8, 4, 1, true, true, unsigned short, 0>"]["bytes_per_launch"]


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=60)
    assert r.returncode == 2 and "one GPU" in r.stderr
