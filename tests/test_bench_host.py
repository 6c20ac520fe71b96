"""Host logic of bench.py: the roofline arithmetic and the choice of the
dominant kernel, the counter-summary lookup and its construction from
rocprofv3 CSV output, and the single-GPU guard (no GPU needed)."""
import csv
import json
import os
import subprocess
import sys

import bench
from workloads import planted

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def fake_plan(tiled=True):
    return {"W": 16, "G1": 4, "G2": 4, "fused": 1, "NB": 256, "esize": 2, "parts1": 1, "parts2": 1,
            "T1R": 1954 if tiled else 0, "T1cb": 13, "T1grid": 256, "T2R": 1954 if tiled else 0, "T2cb": 13,
            "T2grid": 256, "T1un": 1, "T2un": 1}


def test_roofline_entry_dominant_kernel_and_arithmetic():
    A = planted(300, 200, 150, 6, 1)
    s = 16
    b1 = 4 * (A.m + 1) + 5 * A.nnz + 4 * s * (A.n + A.m)
    b2 = 4 * (A.n + 1) + 5 * A.nnz + 4 * s * (A.m + A.n)
    # second product dominant
    rf = bench.roofline_entry(A, s, 65521, [10.0, 20.0, 0.0], fake_plan())
    assert rf["bytes_per_launch"] == b2 and rf["avg_launch_us"] == 20.0
    assert abs(rf["achieved"] - round(b2 / 20e-6 / 1e9, 1)) < 1e-9
    assert abs(rf["frac"] - round(rf["achieved"] / 8000.0, 4)) < 1e-4
    assert rf["kernel"].startswith("k_spmm_tiled<16, unsigned short, false, 1>")
    assert rf["other_product"]["bytes_per_launch"] == b1
    assert rf["step"]["bytes"] == b1 + b2 and rf["step"]["kernel_us"] == 30.0
    # first product dominant; a separate projection counts with the second product
    rf = bench.roofline_entry(A, s, 65521, [25.0, 10.0, 5.0], fake_plan(False))
    assert rf["bytes_per_launch"] == b1 and rf["avg_launch_us"] == 25.0
    assert rf["kernel"].startswith("k_spmm_split<16, 4, ACC, true, false, unsigned short, 0>")
    assert rf["other_product"]["avg_launch_us"] == 15.0
    json.dumps(rf)


def test_product_kernel_names():
    n, src, _ = bench.product_kernel(fake_plan(), 1, 16, 2**31 - 1)
    assert n == "k_spmm_tiled<16, unsigned short, true, 0>" and src.endswith("spmm_tiled.hip")
    n, src, _ = bench.product_kernel(dict(fake_plan(False), esize=4), 2, 16, 2**31 - 1)
    assert n == "k_spmm_split<16, 4, ACC, false, true, unsigned int, 0>" and src.endswith("spmm.hip")


def _write_csv(path, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for r in rows:
            w.writerow(r)


def test_traffic_from_and_lookup(tmp_path, monkeypatch):
    """traffic.json built from two counter runs: the copy of 256 MiB calibrates both counters, each kernel's
    per-dispatch average is scaled; the lookup refuses another revision of the source."""
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    for rel, text in (("paper_0704_2351_amd/csrc/spmm_tiled.hip", "tiled v1"),
                      ("paper_0704_2351_amd/csrc/spmm.hip", "split v1")):
        (tmp_path / rel).parent.mkdir(parents=True, exist_ok=True)
        (tmp_path / rel).write_text(text)
    (tmp_path / "profiles").mkdir()
    kt = ("void bwr::(anonymous namespace)::k_spmm_tiled<16, unsigned short, false, 1>(long, long, int, "
          "unsigned int const*, bwr::ModP)")
    ks = "void bwr::(anonymous namespace)::k_spmm_split<16, 4, 1, true, false, unsigned short, 0>(long, bwr::ModP)"
    cp = "void at::native::elementwise_kernel<128, 4, copy>(int, at::native::copy_kernel)"
    big = 256 * 1024
    _write_csv(str(tmp_path / "f" / "run_counter_collection.csv"),
               [{"Kernel_Name": kt, "Counter_Name": "FETCH_SIZE", "Counter_Value": 1000.0},
                {"Kernel_Name": kt, "Counter_Name": "FETCH_SIZE", "Counter_Value": 3000.0},
                {"Kernel_Name": ks, "Counter_Name": "FETCH_SIZE", "Counter_Value": 500.0},
                {"Kernel_Name": cp, "Counter_Name": "FETCH_SIZE", "Counter_Value": big / 2}])
    _write_csv(str(tmp_path / "w" / "run_counter_collection.csv"),
               [{"Kernel_Name": kt, "Counter_Name": "WRITE_SIZE", "Counter_Value": 100.0},
                {"Kernel_Name": kt, "Counter_Name": "WRITE_SIZE", "Counter_Value": 100.0},
                {"Kernel_Name": ks, "Counter_Name": "WRITE_SIZE", "Counter_Value": 50.0},
                {"Kernel_Name": cp, "Counter_Name": "WRITE_SIZE", "Counter_Value": big}])
    rec = bench.traffic_from(str(tmp_path / "f"), str(tmp_path / "w"), str(tmp_path / "profiles" / "traffic.json"))
    assert rec["fetch_factor"] == 2.0 and rec["write_factor"] == 1.0
    assert bench.kernel_traffic("k_spmm_tiled<16, unsigned short, false, 1>") == 1024 * (2000 * 2 + 100)
    assert bench.kernel_traffic("k_spmm_split<16, 4, ACC, true, false, unsigned short, 0>") == 1024 * (500 * 2 + 50)
    assert bench.kernel_traffic("k_spmm_tiled<16, unsigned short, false, 0>") is None  # not measured
    (tmp_path / "paper_0704_2351_amd/csrc/spmm_tiled.hip").write_text("tiled v2")
    assert bench.kernel_traffic("k_spmm_tiled<16, unsigned short, false, 1>") is None  # another revision
    assert bench.kernel_traffic("k_spmm_split<16, 4, ACC, true, false, unsigned short, 0>") == 1024 * 1050


def test_committed_traffic_record_belongs_to_the_sources():
    """The committed counter summary is current for every source it names (else the bench reports traffic
    null), and it holds the kernels of the default workload's plan."""
    rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    assert "sources" in rec and rec["kernels"]
    for src, digest in rec["sources"].items():
        assert bench._source_digest(src) == digest, src


def test_cpu_info():
    model, threads = bench.cpu_info()
    assert isinstance(model, str) and threads >= 1


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=60)
    assert r.returncode == 2 and "one GPU" in r.stderr
