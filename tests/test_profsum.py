"""Host logic of the rocprofv3 summaries (no GPU): kernel names, per-kernel
aggregation and the copy-probe scaling of the HBM counters."""
import csv

import pytest

from paper_2207_14208_amd import profsum


def _write(path, header, rows):
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(header)
        w.writerows(rows)


def test_short_names_keep_template_arguments_and_drop_parameters():
    assert profsum._short("void bcmg::k_rb_sweep<3, double>(bcmg::Desc const*, int)") == "k_rb_sweep<3, double>"
    assert profsum._short("k_norm_finish(NormRange const*, int)") == "k_norm_finish"
    assert profsum._short("__amd_rocclr_copyBuffer") == "__amd_rocclr_copyBuffer"


def test_trace_table_groups_by_kernel_and_grid(tmp_path):
    hdr = ["Kernel_Name", "Grid_Size_X", "Start_Timestamp", "End_Timestamp"]
    _write(tmp_path / "t_kernel_trace.csv", hdr, [
        ["void k_a<3, double>(int)", 1024, 0, 4000],
        ["void k_a<3, double>(int)", 1024, 10, 2010],
        ["void k_a<3, double>(int)", 256, 0, 1000],
        ["void k_b(int)", 64, 0, 1000],
    ])
    rows, tot_ms = profsum.trace_table(str(tmp_path), top=10)
    assert tot_ms == pytest.approx(8000 / 1e6)
    assert rows[0] == ("k_a<3, double>", 1024, 2, pytest.approx(3.0), pytest.approx(75.0))
    assert {(k, g) for k, g, *_ in rows[1:]} == {("k_a<3, double>", 256), ("k_b", 64)}


def test_traffic_scales_counters_by_the_copy_probe(tmp_path):
    # a 1 MiB copy whose FETCH_SIZE reads 512 KiB and WRITE_SIZE 1024 KiB:
    # factors 2 and 1, so a kernel reading 100 KiB and writing 30 KiB moves
    # 230 KiB per launch
    hdr = ["Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"]
    fd, wd = tmp_path / "f", tmp_path / "w"
    fd.mkdir()
    wd.mkdir()
    _write(fd / "c_counter_collection.csv", hdr, [
        ["elementwise_copy_kernel(int)", 4096, "FETCH_SIZE", 512.0],
        ["void k_rb_sweep<3, double>(int)", 2048, "FETCH_SIZE", 90.0],
        ["void k_rb_sweep<3, double>(int)", 2048, "FETCH_SIZE", 110.0],
        ["void k_rb_sweep<3, double>(int)", 512, "FETCH_SIZE", 7.0],
    ])
    _write(wd / "c_counter_collection.csv", hdr, [
        ["elementwise_copy_kernel(int)", 4096, "WRITE_SIZE", 1024.0],
        ["void k_rb_sweep<3, double>(int)", 2048, "WRITE_SIZE", 30.0],
        ["void k_rb_sweep<3, double>(int)", 512, "WRITE_SIZE", 2.0],
    ])
    t = profsum.traffic(str(fd), str(wd), "k_rb_sweep<3, double>", 0, 1 << 20)
    assert t["grid"] == 2048 and t["dispatches"] == [2, 1]
    assert t["fetch_scale"] == pytest.approx(2.0) and t["write_scale"] == pytest.approx(1.0)
    assert t["bytes_per_launch"] == pytest.approx(230.0 * 1024)


def test_copy_probe_is_the_first_large_copy(tmp_path):
    # the probe copy (dispatch 2) comes before a larger upload of the inputs
    # (dispatch 9, same copy kernel): the factors come from the probe
    hdr = ["Dispatch_Id", "Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"]
    fd, wd = tmp_path / "f", tmp_path / "w"
    fd.mkdir()
    wd.mkdir()
    _write(fd / "c_counter_collection.csv", hdr, [
        [1, "fill_kernel(int)", 4096, "FETCH_SIZE", 0.0],
        [2, "__amd_rocclr_copyBuffer", 4096, "FETCH_SIZE", 512.0],
        [5, "void k_rb_sweep<3, float>(int)", 2048, "FETCH_SIZE", 100.0],
        [9, "__amd_rocclr_copyBuffer", 4096, "FETCH_SIZE", 2048.0],
        [12, "__amd_rocclr_copyBuffer", 4096, "FETCH_SIZE", 1.5],
    ])
    _write(wd / "c_counter_collection.csv", hdr, [
        [2, "__amd_rocclr_copyBuffer", 4096, "WRITE_SIZE", 1024.0],
        [5, "void k_rb_sweep<3, float>(int)", 2048, "WRITE_SIZE", 30.0],
        [9, "__amd_rocclr_copyBuffer", 4096, "WRITE_SIZE", 4096.0],
    ])
    t = profsum.traffic(str(fd), str(wd), "k_rb_sweep<3, float>", 0, 1 << 20)
    assert t["copy_fetch_kib"] == 512.0 and t["copy_write_kib"] == 1024.0
    assert t["bytes_per_launch"] == pytest.approx(230.0 * 1024)


def test_marker_ranges_group_and_count_kernel_time_inside(tmp_path):
    # two host checks of a solve and a setup range; kernels count toward a
    # range only when they start and end inside it
    _write(tmp_path / "m_marker_api_trace.csv",
           ["Domain", "Function", "Process_Id", "Thread_Id", "Correlation_Id", "Start_Timestamp", "End_Timestamp"], [
               ["MARKER_CORE_RANGE_API", "bcmg_setup 3D N=8", 1, 1, 1, 0, 1_000_000],
               ["MARKER_CORE_RANGE_API", "bcmg_solve", 1, 1, 2, 2_000_000, 9_000_000],
               ["MARKER_CORE_RANGE_API", "cycles 1..1", 1, 1, 3, 2_100_000, 3_000_000],
               ["MARKER_CORE_RANGE_API", "cycles 2..9", 1, 1, 4, 3_000_000, 8_900_000],
           ])
    _write(tmp_path / "m_kernel_trace.csv", ["Kernel_Name", "Grid_Size_X", "Start_Timestamp", "End_Timestamp"], [
        ["k_classify_a", 64, 100_000, 300_000],
        ["k_rb_sweep<3, double>", 64, 2_200_000, 2_700_000],
        ["k_rb_sweep<3, double>", 64, 3_500_000, 4_500_000],
        ["k_rb_sweep<3, double>", 64, 8_800_000, 9_500_000],  # ends after both ranges
    ])
    rows = {k: (n, host, kern) for k, n, host, kern in profsum.marker_table(str(tmp_path))}
    assert rows["bcmg_setup 3D N=8"] == (1, 1.0, 0.2)
    assert rows["bcmg_solve"] == (1, 7.0, 1.5)
    n, host, kern = rows["cycles a..b (one host check)"]
    assert n == 2 and abs(host - 6.8) < 1e-12 and abs(kern - 1.5) < 1e-12


def test_last_dispatches_average_the_final_burst(tmp_path):
    # dispatches out of order in the file: the last two by start time are
    # the 5 us and 7 us ones; another grid and another kernel are ignored
    hdr = ["Kernel_Name", "Grid_Size_X", "Start_Timestamp", "End_Timestamp"]
    _write(tmp_path / "t_kernel_trace.csv", hdr, [
        ["void k_a<3>(int)", 1024, 300, 7300],
        ["void k_a<3>(int)", 1024, 0, 20000],
        ["void k_a<3>(int)", 1024, 200, 5200],
        ["void k_a<3>(int)", 512, 900, 9900],
        ["void k_b(int)", 1024, 1000, 90000],
    ])
    avg, n = profsum.last_dispatches_us(str(tmp_path), "k_a<3>", 1024, 2)
    assert n == 2 and avg == pytest.approx(6.0)
    avg, n = profsum.last_dispatches_us(str(tmp_path), "k_a<3>", 1024, 10)
    assert n == 3 and avg == pytest.approx((20.0 + 5.0 + 7.0) / 3)
