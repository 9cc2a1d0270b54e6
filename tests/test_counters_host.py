"""Host logic of the counter summaries (no GPU): which dispatches make up the last R fine-level residuals when
the divergence (and the gradient) launch once per tile-size class, and the scaling of the HBM counters by a
plain copy of known size."""
import csv
import json
import os

import pytest

from paper_1806_11456_amd import counters


def _row(i, name, value, grid=256):
    return {"Dispatch_Id": str(i), "Kernel_Name": f"void {name}<double, 1, 256>(LevelDevT<double>, ...)",
            "Counter_Value": str(value), "Grid_Size": str(grid)}


def _residual(rows, start, div_launches, value):
    """One residual's dispatches: trace, gradient (per class), flux, divergence (per class)."""
    i = start
    for name, n in (("k_trace", 1), ("k_grad", div_launches), ("k_face2c", 1), ("k_div", div_launches)):
        for _ in range(n):
            rows.append(_row(i, name, value))
            i += 1
    return i


def test_last_residuals_with_class_split_launches():
    rows = []
    i = 0
    rows.append(_row(i, "k_fill", 1.0))  # setup work before the residuals is not counted
    i += 1
    for r in range(5):
        # residual r: every dispatch counts r + 1, divergence and gradient in 3 launches
        i = _residual(rows, i, 3, float(r + 1))
    got = counters._last_residuals(rows, 2)
    # the last two residuals: 1 trace + 3 gradient + 1 flux + 3 divergence dispatches each
    assert len(got) == 16
    assert sorted({float(r["Counter_Value"]) for r in got}) == [4.0, 5.0]
    with pytest.raises(SystemExit):
        counters._last_residuals(rows, 5)  # only four residual ends follow an earlier one


def test_last_residuals_order_by_dispatch_id():
    rows = []
    i = _residual(rows, 0, 1, 1.0)
    i = _residual(rows, i, 2, 2.0)
    i = _residual(rows, i, 1, 3.0)
    rows.reverse()  # the CSV order is not the dispatch order
    got = counters._last_residuals(rows, 1)
    assert [r["Kernel_Name"].split("<")[0] for r in sorted(got, key=lambda r: int(r["Dispatch_Id"]))] == [
        "void k_trace", "void k_grad", "void k_face2c", "void k_div"]
    assert {float(r["Counter_Value"]) for r in got} == {3.0}


def test_residual_traffic_scales_by_the_copy(tmp_path):
    # a 1 MiB copy reads FETCH_SIZE = 512 KiB and writes WRITE_SIZE = 1024 KiB: scales 2 and 1
    def write(d, per_dispatch):
        os.makedirs(d)
        rows = [{"Dispatch_Id": "0", "Kernel_Name": "__amd_rocclr_copyBuffer", "Counter_Value": str(per_dispatch[0]),
                 "Grid_Size": "1048576"}]
        i = 1
        for r in range(3):
            i = _residual(rows, i, 2, per_dispatch[1])
        with open(os.path.join(d, "run_counter_collection.csv"), "w", newline="") as f:
            w = csv.DictWriter(f, fieldnames=list(rows[0]))
            w.writeheader()
            w.writerows(rows)
    write(tmp_path / "f", (512.0, 10.0))
    write(tmp_path / "w", (1024.0, 4.0))
    out = tmp_path / "t.json"
    counters.residual_traffic(str(tmp_path / "f"), str(tmp_path / "w"), 2, 1, str(out), "cmd", 1000.0)
    d = json.loads(out.read_text())
    assert d["fetch_scale"] == pytest.approx(2.0) and d["write_scale"] == pytest.approx(1.0)
    # per residual: 6 dispatches x (10 KiB x 2 + 4 KiB x 1) = 144 KiB
    assert d["traffic_bytes_per_residual"] == pytest.approx(6 * (10 * 2 + 4) * 1024.0)
    assert d["per_kernel_bytes"]["k_div"]["fetch"] == pytest.approx(2 * 10 * 2 * 1024.0)


def test_source_hash_covers_only_the_residual_kernels():
    h = counters.source_hash()
    assert len(h) == 64
    assert set(counters.RESIDUAL_SOURCES) == {"device.h", "kernels_elem.inc", "kernels_face.inc"}
