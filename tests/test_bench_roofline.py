"""The benchmark's roofline bookkeeping (host logic, no GPU).

The JSON line's `roofline` comes from the in-library profiler's per-launch algorithmic bytes and flops
and the measured time; `traffic` and the matrix-core counter fields come from profiles/traffic.json only
while its record matches the kernel's source hash and the tuned variant.  These tests build fake
profiler records and check the arithmetic, the bound label and the record matching.
"""
import importlib.util
import json
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _record(name, ms, gb, tflop, launches=4):
    return {"name": name, "launches": launches, "total_ms": ms * launches, "bytes": gb * 1e9 * launches,
            "stored_bytes": gb * 1e9 * launches, "flops": tflop * 1e12 * launches}


def test_hbm_bound_label_and_fractions(bench):
    r = bench.roofline(_record("down_fp32_rt1_s2", 0.5, 2.0, 0.002), "fp32", None, "nowhere")
    assert r["bound"] == "hbm" and r["unit"] == "GB/s"
    assert r["achieved"] == pytest.approx(4000.0, rel=1e-6)           # 2 GB in 0.5 ms
    assert r["frac"] == pytest.approx(0.5, rel=1e-6)                  # of 8 TB/s
    assert r["traffic"] is None                                        # no record for this workload


def test_compute_bound_label_uses_the_precision_peak(bench):
    r = bench.roofline(_record("middle_mfma_fp32", 10.0, 1.0, 1.0), "fp32", None, "nowhere")
    assert r["bound"] == "mfma" and r["peak"] == 157.3
    assert r["achieved"] == pytest.approx(100.0, rel=1e-6)            # 1 TFLOP in 10 ms
    s = bench.roofline(_record("middle_fp16x3", 10.0, 1.0, 10.0), "fp16x3", None, "nowhere")
    assert s["peak"] == 2500.0 and s["bound"] == "mfma"
    assert s["frac"] == pytest.approx(0.4, rel=1e-6)


def test_counter_record_requires_matching_source_and_variant(bench):
    with open(os.path.join(ROOT, "profiles", "traffic.json")) as fh:
        data = json.load(fh)
    for key, rec in data.items():
        workload, kernel = key.split("/", 1)
        if kernel == "id_kernel":
            continue
        files = bench.kernel_sources(kernel)
        assert set(rec["source_files"]) == set(files), key
        current = rec["source_sha"] == bench.source_sha(files)
        variant = rec["variants"][0] if rec.get("variants") else None
        got = bench.counter_record(kernel, variant, workload)
        assert (got is not None) == current, key
        if rec.get("variants"):
            assert bench.counter_record(kernel, -1, workload) is None     # another variant: no record
        if got is not None:
            assert bench.traffic_for(kernel, variant, workload) == rec["hbm_bytes_per_launch"]


def test_counter_fields_join_the_roofline(bench):
    with open(os.path.join(ROOT, "profiles", "traffic.json")) as fh:
        data = json.load(fh)
    rec = data.get("fio512x64/down_dense_fp16x3_s2")
    if rec is None or rec["source_sha"] != bench.source_sha(bench.kernel_sources("down_dense_fp16x3_s2")):
        pytest.skip("no current counter record for the dense down pass")
    r = bench.roofline(_record("down_dense_fp16x3_s2", 2.0, 9.0, 2.0), "fp16x3", rec["variants"][0], "fio512x64")
    assert r["traffic"] == rec["hbm_bytes_per_launch"]
    assert r["mfma_util_counters"] == rec["mfma_util"]
    assert r["mfma_TFLOPs_counters"] == pytest.approx(rec["mfma_flops_per_launch"] / 2e-3 / 1e12, rel=1e-3)


def test_id_roofline_traffic_only_for_a_matching_record(bench):
    st = {"id_ms": 1000.0, "id_flops": 7.86e12, "id_bytes": 8e11}
    r = bench.id_roofline(st, "nowhere")
    assert r["frac_fp64"] == pytest.approx(0.1, rel=1e-6)            # 7.86 TFLOP in 1 s of 78.6 TFLOP/s
    assert r["frac_hbm"] == pytest.approx(0.1, rel=1e-6)             # 0.8 TB in 1 s of 8 TB/s
    assert r["traffic"] is None
