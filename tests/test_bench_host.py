"""Host-side logic of the measurement script (no GPU): the method's bytes per
estimate, kernel-name handling, the copy-calibrated counter summaries, the
kernel-trace summary, the step records and the row relabelling."""
import csv
import json
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
import workloads as w  # noqa: E402


def test_method_bytes_of_the_bench_workload():
    # one CSR pass: 8 B per entry + row pointers; the sketch step reads and
    # writes the block and the accumulator (16 B per element), the
    # quadratic-form step reads and writes the block and reads X (12 B):
    # 1024^2 grid, 5,238,784 entries, 20 + 20 columns, degree 80
    n, nnz = 1 << 20, 5238784
    a = 8 * nnz + 4 * (n + 1)
    assert a == 46104580
    sketch = a + 16 * n * 20
    quad = a + 12 * n * 40
    assert round(sketch / 1e6, 1) == 381.6 and round(quad / 1e6, 1) == 549.4
    total = bench.method_bytes_per_estimate(n, nnz, 80, 20, 20)
    assert total == pytest.approx(80 * (sketch + quad), rel=1e-15)
    assert round(total / 1e9, 2) == 74.49


def test_short_kernel_names():
    f = bench.short_kernel_name
    assert f("void ld::(anonymous namespace)::step_kernel<float, 4, 3, false, 2, 256, 5>(int, int const*, "
             "float const*)") == "step_kernel<float, 4, 3, false, 2, 256, 5>"
    assert f("ld::chol_factor_kernel(double const*, int, double*, double*, int*)") == "chol_factor_kernel"
    assert f("void ld::adjoint_dia_kernel<float, 4, 8, 5, 4>(int, int const*)") == \
        "adjoint_dia_kernel<float, 4, 8, 5, 4>"
    assert f("__amd_rocclr_copyBuffer") == "__amd_rocclr_copyBuffer"


def _write_counters(d, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "b_counter_collection.csv"), "w", newline="") as fh:
        wr = csv.writer(fh)
        wr.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        for r in rows:
            wr.writerow(r)


def test_traffic_summary_scales_by_the_copy(tmp_path):
    # the copy reads and writes 1 GiB; FETCH_SIZE reports half of the bytes
    # read (x2), WRITE_SIZE all of them (x1).  A step kernel with two
    # dispatches, each reported in two counter instances that add up
    copy = "void at::native::copy_kernel(float const*)"
    step = "void ld::(anonymous namespace)::step_kernel<float, 4, 3, false, 2, 256, 5>(int)"
    gib_kib = (1 << 30) / 1024
    _write_counters(tmp_path / "cf", [(1, copy, "FETCH_SIZE", gib_kib / 2)])
    _write_counters(tmp_path / "cw", [(1, copy, "WRITE_SIZE", gib_kib)])
    _write_counters(tmp_path / "f", [(2, step, "FETCH_SIZE", 30000.0), (2, step, "FETCH_SIZE", 20000.0),
                                     (3, step, "FETCH_SIZE", 40000.0), (3, step, "FETCH_SIZE", 30000.0)])
    _write_counters(tmp_path / "w", [(2, step, "WRITE_SIZE", 80000.0), (3, step, "WRITE_SIZE", 80000.0)])
    log = tmp_path / "line.log"
    alg = 200e6
    log.write_text("noise\n" + json.dumps({"kernels": {"quadform": {"kernel": "step_kernel",
                                                                    "bytes_per_launch": alg}}}) + "\n")
    out = bench.traffic_summary([str(tmp_path / x) for x in ("f", "w", "cf", "cw")], str(log))
    read_mb = 60000.0 * 2 * 1024 / 1e6          # mean over dispatches, x2, KiB -> MB
    write_mb = 80000.0 * 1024 / 1e6
    row = [l for l in out.splitlines() if l.startswith("| step_kernel")][0].split("|")
    assert float(row[2]) == pytest.approx(read_mb, abs=0.05)
    assert float(row[3]) == pytest.approx(write_mb, abs=0.05)
    assert float(row[5]) == pytest.approx(alg / 1e6, abs=0.05)
    assert float(row[6]) == pytest.approx((read_mb + write_mb) / (alg / 1e6), abs=0.005)
    blob = json.loads(out.split("```json", 1)[1].split("```", 1)[0])
    assert blob["source_hash"] == bench.source_hash()
    assert blob["traffic_MB_per_launch"]["step_kernel<float, 4, 3, false, 2, 256, 5>"] == \
        pytest.approx(read_mb + write_mb, abs=1e-3)
    assert not any(k.startswith("at::") for k in blob["traffic_MB_per_launch"])   # torch's copy left out


def test_stats_summary_table(tmp_path):
    with open(tmp_path / "b_kernel_stats.csv", "w", newline="") as fh:
        wr = csv.writer(fh)
        wr.writerow(["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage"])
        wr.writerow(["void ld::(anonymous namespace)::dia_flat_kernel<float, 4, 0, 5>(int)", 80, 2400000, 30000,
                     41.5])
    out = bench.stats_summary(str(tmp_path))
    assert "| dia_flat_kernel<float, 4, 0, 5> | 80 | 30.00 | 2.40 | 41.50 |" in out


def test_step_records_from_library_timings():
    st = {"ms_steps1": 2.4, "launches1": 80, "bytes1": 80 * 178.3e6, "ms_steps23": 2.8, "launches23": 80,
          "bytes23": 80 * 169.9e6, "dia_diagonals": 5}
    k = bench.kernel_records(st)
    assert k["sketch_horner"]["kernel"] == "dia_flat_kernel" and k["quadform"]["kernel"] == "step_kernel"
    assert k["sketch_horner"]["avg_us"] == pytest.approx(30.0)
    assert k["quadform"]["GBps"] == pytest.approx(169.9e6 / 35e-6 / 1e9)
    st["dia_diagonals"] = 0
    assert bench.kernel_records(st)["sketch_horner"]["kernel"] == "step_kernel"


@pytest.mark.parametrize("order", ["rcm", "degree", "random"])
def test_relabelling_is_a_symmetric_permutation(order):
    csr = w.grid_laplacian_2d(9, 0.3)
    row_ptr, col_idx, val, n = bench.relabel(csr, order)
    A = w.to_scipy(csr).toarray()
    B = w.to_scipy((row_ptr, col_idx, val, n)).toarray()
    np.testing.assert_allclose(np.linalg.eigvalsh(B), np.linalg.eigvalsh(A), rtol=1e-13, atol=1e-13)
    assert all(np.all(np.diff(col_idx[row_ptr[i]:row_ptr[i + 1]]) > 0) for i in range(n))
    if order == "degree":
        assert np.all(np.diff(np.diff(row_ptr)) <= 0)


def test_bench_runs_on_one_gpu_only():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=120)
    assert out.returncode != 0 and "exactly one GPU" in (out.stdout + out.stderr)


def test_traffic_summary_counts_row_range_dispatches(tmp_path):
    # a quadratic-form step that runs as 4 dispatches over row ranges: the
    # counters per dispatch times 4 are the bytes of one library launch
    copy = "void at::native::copy_kernel(float const*)"
    first = "void ld::(anonymous namespace)::step_kernel<float, 4, 3, true, 2, 256, 5>(int)"
    rest = "void ld::(anonymous namespace)::step_kernel<float, 4, 3, false, 2, 256, 5>(int)"
    gib_kib = (1 << 30) / 1024
    _write_counters(tmp_path / "cf", [(1, copy, "FETCH_SIZE", gib_kib / 2)])
    _write_counters(tmp_path / "cw", [(1, copy, "WRITE_SIZE", gib_kib)])
    _write_counters(tmp_path / "f", [(2, first, "FETCH_SIZE", 500.0)] +
                    [(3 + i, rest, "FETCH_SIZE", 1000.0) for i in range(8)])
    _write_counters(tmp_path / "w", [(2, first, "WRITE_SIZE", 250.0)] +
                    [(3 + i, rest, "WRITE_SIZE", 500.0) for i in range(8)])
    log = tmp_path / "line.log"
    alg = 9e6
    log.write_text(json.dumps({"kernels": {"quadform": {"kernel": "step_kernel", "bytes_per_launch": alg,
                                                        "dispatches_per_launch": 4}}}) + "\n")
    out = bench.traffic_summary([str(tmp_path / x) for x in ("f", "w", "cf", "cw")], str(log))
    blob = json.loads(out.split("```json", 1)[1].split("```", 1)[0])["traffic_MB_per_launch"]
    per_launch = 4 * (1000.0 * 2 + 500.0) * 1024 / 1e6
    assert blob["step_kernel<float, 4, 3, false, 2, 256, 5>"] == pytest.approx(per_launch, abs=1e-3)
    assert blob["step_kernel<float, 4, 3, true, 2, 256, 5>"] == pytest.approx(per_launch / 2, abs=1e-3)
    row = [l for l in out.splitlines() if l.startswith("| step_kernel<float, 4, 3, false")][0].split("|")
    assert float(row[6]) == pytest.approx(per_launch / (alg / 1e6), abs=0.005)
