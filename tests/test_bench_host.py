"""Host-side logic of bench.py: roofline arithmetic, the family table and the
stored traffic figure's source pin (no GPU)."""
import importlib.util
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_host", os.path.join(ROOT, "bench.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


def _fam(launches, ms, flops, nbytes):
    return {"launches": launches, "ms": ms, "flops": flops, "bytes": nbytes}


def test_product_roofline_per_precision(bench):
    # 10 FP32 launches of 1 GFLOP in 0.1 ms total: 100 TFLOP/s against 157.3;
    # 2 FP64 launches of 1 GFLOP in 0.04 ms total: 50 TFLOP/s against 78.6
    fams = {"product": _fam(12, 0.14, 12e9, 12e8),
            "product_fp32": _fam(10, 0.1, 10e9, 10e8),
            "product_fp64": _fam(2, 0.04, 2e9, 2e8),
            "product_bf16": _fam(0, 0.0, 0.0, 0.0)}
    r = bench.product_roofline(fams, "fp32")
    byp = r["by_precision"]
    assert set(byp) == {"fp32", "fp64"}
    assert byp["fp32"]["achieved_tflops"] == pytest.approx(100.0)
    assert byp["fp32"]["frac_mfma"] == pytest.approx(100.0 / 157.3)
    assert byp["fp64"]["achieved_tflops"] == pytest.approx(50.0)
    assert byp["fp64"]["frac_mfma"] == pytest.approx(50.0 / 78.6)
    # the aggregate: 12 GFLOP in 0.14 ms against the phase precision's peak
    assert r["achieved_tflops"] == pytest.approx(12e9 / 0.14e-3 / 1e12)
    assert r["peak_tflops"] == pytest.approx(157.3)
    assert bench.product_roofline({"product": _fam(0, 0.0, 0.0, 0.0)}, "fp32") is None


def test_kernel_table_keeps_families_only(bench):
    fams = {f: _fam(1, 1.0, 1e9, 1e6) for f in bench.FAMILIES}
    fams["product_fp32"] = _fam(1, 1.0, 1e9, 1e6)
    fams["gram"] = _fam(0, 0.0, 0.0, 0.0)
    t = bench.kernels_table(fams)
    assert "product_fp32" not in t and "gram" not in t
    assert set(t) == set(bench.FAMILIES) - {"gram"}
    assert t["product"] == {"launches": 1, "ms": 1.0, "gflop": 1.0, "gbyte": 0.001}


def test_traffic_pin_follows_sources(bench):
    # the stored figure is reported only while the kernel sources hash to the
    # value recorded with it
    t = bench.TRAFFIC[("n4000_mixed_iid", "product")]
    assert bench.measured_traffic("n4000_mixed_iid", "product") in (None, t["bytes"])
    assert bench.measured_traffic("no_such_workload", "product") is None
    assert os.path.exists(os.path.join(ROOT, t["profile"]))
    for f in t["files"]:
        assert os.path.exists(os.path.join(ROOT, f)), f


def test_rebuild_roofline_bound_follows_intensity(bench):
    # a rebuild from hundreds of pairs is compute-bound, from a few HBM-bound
    big = bench.roofline({"rebuild": _fam(1, 0.3, 4000.0 ** 2 * 370, 8 * 4000.0 ** 2)}, "fp64")
    small = bench.roofline({"rebuild": _fam(1, 0.05, 4000.0 ** 2 * 40, 8 * 4000.0 ** 2)}, "fp64")
    assert big["bound"] == "alu" and small["bound"] == "hbm"


def test_product_roofline_takes_dominant_precision(bench):
    fams = {"product": _fam(20, 2.0, 20 * 1.5e9, 20 * 1.3e8),
            "product_fp64": _fam(10, 1.2, 10 * 1.5e9, 10 * 1.3e8),
            "product_fp32": _fam(10, 0.8, 10 * 1.5e9, 10 * 0.65e8),
            "rr": _fam(5, 0.5, 1e6, 1e5)}
    r = bench.roofline(fams, "fp32")
    assert r["kernel"] == "product" and r["precision"] == "fp64"
    assert abs(r["peak"] - 78.6) < 1e-9
    assert abs(r["achieved"] - 1.5e9 / 0.12e-3 / 1e12) < 1e-9
