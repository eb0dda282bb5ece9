"""Host logic of bench.py (no GPU): the roofline record built from the
library's per-kernel timings, the traffic lookup guarded by the kernel source
hash, and the counter summaries written from rocprofv3 CSV files."""
import csv
import json
import os

import pytest

import bench


def _stat(name, launches, ms, flops=0.0, bytes_=0.0):
    return {"name": name, "launches": launches, "ms": ms, "flops": flops, "bytes": bytes_}


def test_roofline_takes_the_kernel_with_the_largest_summed_time():
    stats = [_stat("formA", 3, 270.0, flops=3 * 4 * 2000.0 ** 3 * 256),
             _stat(bench.TRAFFIC_CLASS, 57, 392.0, flops=57 * 4.49e11),
             _stat("lu_panel", 96, 88.0, bytes_=96 * 3.5e8)]
    r = bench.kernel_roofline(stats)
    assert r["kernel"] == bench.TRAFFIC_CLASS and r["bound"] == "mfma"
    achieved = 57 * 4.49e11 / 0.392 / 1e12
    assert abs(r["achieved"] - achieved) < 1e-9 * achieved
    assert abs(r["frac"] - achieved / 78.6) < 1e-12
    assert abs(r["avg_launch_us"] - 392.0e3 / 57) < 1e-9
    assert set(r["all_kernels"]) == {"formA", bench.TRAFFIC_CLASS, "lu_panel"}


def test_roofline_of_vector_unit_and_memory_kernels():
    r = bench.kernel_roofline([_stat("sigma_contract", 5, 300.0, flops=5 * 8.9e11)])
    assert r["bound"] == "alu" and r["peak"] == 78.6
    r = bench.kernel_roofline([_stat("symmetrize", 1, 13.0, bytes_=6.6e10)])
    assert r["bound"] == "hbm" and r["unit"] == "GB/s"
    assert abs(r["achieved"] - 6.6e10 / 0.013 / 1e9) < 1e-6
    assert r["traffic"] is None
    assert bench.kernel_roofline([_stat("idle", 1, 0.0)]) is None


def test_stored_traffic_needs_the_same_kernel_sources(tmp_path, monkeypatch):
    f = tmp_path / "t.json"
    f.write_text(json.dumps({"kernel": bench.TRAFFIC_KERNEL, "kernel_source_sha256_16": bench.kernel_source_hash(),
                             "bytes_per_launch": 123.0}))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.stored_traffic() == 123.0
    f.write_text(json.dumps({"kernel": bench.TRAFFIC_KERNEL, "kernel_source_sha256_16": "0" * 16,
                             "bytes_per_launch": 123.0}))
    assert bench.stored_traffic() is None
    f.write_text(json.dumps({"kernel": "another kernel", "kernel_source_sha256_16": bench.kernel_source_hash(),
                             "bytes_per_launch": 123.0}))
    assert bench.stored_traffic() is None


def _write_csv(path, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=list(rows[0]))
        w.writeheader()
        w.writerows(rows)


def test_counter_summaries(tmp_path):
    """FETCH_SIZE / WRITE_SIZE are averaged per kernel and scaled by the copy
    calibration (a 1 GiB pass that reads half its bytes in FETCH_SIZE), and
    MfmaUtil / MfmaFlopsF64 are averaged per kernel."""
    copy_k = "vectorized_elementwise_kernel<4, AUnaryFunctor<double, double, double, MulFunctor<double> > >"
    dom = "void k_gemm(int) " + bench.TRAFFIC_KERNEL
    gib_kib = bench.COPY_BYTES / 1024.0
    _write_csv(tmp_path / "fetch.csv", [
        {"Kernel_Name": copy_k, "Counter_Name": "FETCH_SIZE", "Counter_Value": gib_kib / 2},
        {"Kernel_Name": dom, "Counter_Name": "FETCH_SIZE", "Counter_Value": 100.0},
        {"Kernel_Name": dom, "Counter_Name": "FETCH_SIZE", "Counter_Value": 300.0}])
    _write_csv(tmp_path / "write.csv", [
        {"Kernel_Name": copy_k, "Counter_Name": "WRITE_SIZE", "Counter_Value": gib_kib},
        {"Kernel_Name": dom, "Counter_Name": "WRITE_SIZE", "Counter_Value": 50.0}])
    out = tmp_path / "t.json"
    bench.summarize_profiles(str(tmp_path / "stats.csv"), str(tmp_path / "fetch.csv"), str(tmp_path / "write.csv"),
                             str(out))
    t = json.loads(out.read_text())
    assert t["fetch_scale"] == pytest.approx(2.0) and t["write_scale"] == pytest.approx(1.0)
    assert t["bytes_per_launch"] == pytest.approx((200.0 * 2.0 + 50.0) * 1024.0)
    assert os.path.exists(tmp_path / "hbm_traffic_chain40_n2000.md")

    _write_csv(tmp_path / "mfma.csv", [
        {"Kernel_Name": dom, "Counter_Name": "MfmaUtil", "Counter_Value": 60.0},
        {"Kernel_Name": dom, "Counter_Name": "MfmaUtil", "Counter_Value": 70.0},
        {"Kernel_Name": dom, "Counter_Name": "MfmaFlopsF64", "Counter_Value": 4.0e11},
        {"Kernel_Name": dom, "Counter_Name": "MfmaFlopsF64", "Counter_Value": 5.0e11},
        {"Kernel_Name": "k_hist", "Counter_Name": "MfmaFlopsF64", "Counter_Value": 0.0}])
    md = tmp_path / "m.md"
    bench.summarize_mfma(str(tmp_path / "mfma.csv"), str(md))
    text = md.read_text()
    assert "| 2 | 65.0 | 4.500e+11 |" in text
    assert "k_hist" not in text  # no matrix-core work


def test_solve_flops_with_A_given():
    """The A route hands the solve A = 1 - v chi0: no 4N^3 product per
    frequency (FP64 8N^3: LU 8/3, forward 4, back 4/3; mixed: the residual
    steps only in FP64)."""
    n3 = 100.0 ** 3
    assert bench.solve_flops(100, 1)["fp64"] == pytest.approx(12 * n3)
    assert bench.solve_flops(100, 1, form_a=False)["fp64"] == pytest.approx(8 * n3)
    f = bench.solve_flops(100, 2, n_ir=3, mixed=True, form_a=False)
    assert f["fp64"] == pytest.approx(2 * 24 * n3) and f["fp32"] == pytest.approx(2 * (8.0 / 3 + 32) * n3)
