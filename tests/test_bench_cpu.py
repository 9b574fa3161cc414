"""Host-side pieces of bench.py: the flop model it prices the roofline with and
the conversion of two profiler counter runs into HBM bytes per launch."""
import csv
import importlib.util
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _counter_csv(path, counter, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for d, name, v in rows:
            # two instances (XCDs) per dispatch, summed by the reader
            w.writerow({"Dispatch_Id": d, "Kernel_Name": name, "Counter_Name": counter, "Counter_Value": v / 2})
            w.writerow({"Dispatch_Id": d, "Kernel_Name": name, "Counter_Name": counter, "Counter_Value": v / 2})


def test_traffic_scales_each_counter_by_the_copy(tmp_path):
    b = _bench()
    fused = "void sgbem::tile_kernel<2, 7, 1, true, double, double, 28, 7, 1, 256>(sgbem::TileArgs, sgbem::TileArgsF)"
    copy_kib = 262144.0
    # the fetch counter reads half of the copy's bytes, the write counter all of them; the fill
    # of the copy's source (dispatch 30) writes as much as the copy (dispatch 31)
    f_rows = [(i, fused, 374.0) for i in range(1, 21)] + [(30, "fill", 0.0), (31, "copy", copy_kib / 2)]
    w_rows = [(i, fused, 8192.0) for i in range(1, 21)] + [(30, "fill", copy_kib), (31, "copy", copy_kib)]
    fp, wp = tmp_path / "f.csv", tmp_path / "w.csv"
    _counter_csv(fp, "FETCH_SIZE", f_rows)
    _counter_csv(wp, "WRITE_SIZE", w_rows)
    out = b.write_traffic(str(fp), str(wp), str(tmp_path / "t.json"))
    assert out["fetch_scale"] == pytest.approx(2.0) and out["write_scale"] == pytest.approx(1.0)
    assert out["bytes_per_launch"] == pytest.approx((2 * 374.0 + 8192.0) * 1024)
    assert out["source_hash"] == b.kernel_source_hash()


def test_traffic_refuses_a_run_without_the_copy(tmp_path):
    b = _bench()
    fused = "void sgbem::tile_kernel<2, 7, 1, true, double, double, 28, 7, 1, 256>(sgbem::TileArgs, sgbem::TileArgsF)"
    fp = tmp_path / "f.csv"
    _counter_csv(fp, "FETCH_SIZE", [(1, fused, 374.0)])
    with pytest.raises(SystemExit):
        b.write_traffic(str(fp), str(fp), str(tmp_path / "t.json"))


def test_wq_flop_model():
    """Per entry (fast form, n_ref = R, Q = 2R(p+1) - 1): (4R+1)Q multiply-adds and
    4R^2 kernel values; at the headline (p = 3, R = 1, upper triangle of N = 1024)
    that is the 174 flops per entry and 91315200 flops per launch the roofline uses."""
    b = _bench()
    assert b.wq_flops_per_entry(3, 1) == 174.0
    assert b.wq_flops_per_entry(3, 1) * 1024 * 1025 / 2 == 91315200.0
    for p, R in [(2, 2), (4, 1), (6, 4)]:
        assert b.wq_flops_per_entry(p, R) > 2 * (4 * R + 1) * (2 * R * (p + 1) - 1)
