"""Host-side logic of bench.py (no GPU): the forward kernel's source hash
ignores comments and whitespace but not code, the binding fractions follow
their definitions, and the served-trace overlap sweep counts the time with
kernels of two or more streams."""
import os
import shutil

import pytest

import bench

CSRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1806_02637_amd", "csrc")


def test_source_hash_sees_code_not_comments(tmp_path):
    for name in bench.FWD_SOURCES:
        shutil.copy(os.path.join(CSRC, name), tmp_path / name)
    h0 = bench.fwd_source_hash(str(tmp_path))
    assert h0 == bench.fwd_source_hash()
    p = tmp_path / "ecc.hip"
    text = p.read_text()
    p.write_text("// a new comment line\n/* and a block\n   comment */\n" + text.replace("\n", "\n  ", 3))
    assert bench.fwd_source_hash(str(tmp_path)) == h0
    p.write_text(text.replace("kWavesPerBlock", "kWavesPerBlock ", 1).replace("const int lane", "const int lane2", 1))
    assert bench.fwd_source_hash(str(tmp_path)) != h0


def test_binding_fractions_follow_their_definitions():
    # one XCD-cycle count of 2e7 at 2 GHz = 10 ms profiled; a 10 ms launch
    kc = {"grbm_gui_active": 8 * 2e7, "profiled_ms": 10.0, "tcp_grbm_gui_active": 8 * 2e7,
          "tcp_tcc_read_req": 1e9, "hbm_bytes_per_launch": 20e9, "sq_insts_valu": 1024 * 2e7 / 4 * 0.5,
          "valu_lane_insts_per_eval": 100.0, "tcp_pending_stall_cycles": 256 * 2e7 * 0.25,
          "probe": {"line_bytes": 128, "l2_random_req_per_s": 250e9, "l2_random_req_per_gather": 1.0}}
    b = bench.binding_fractions(kc, 10.0)
    assert b["clock_ghz"] == pytest.approx(2.0)
    assert b["hbm_measured_gbs"] == pytest.approx(2000.0)
    assert b["hbm_measured_frac"] == pytest.approx(2000.0 / bench.HBM_PEAK_GBS)
    assert b["l2_gbs"] == pytest.approx(1e9 * 128 / 0.01 / 1e9)
    assert b["l2_peak_measured"] == pytest.approx(250e9 * 128 / 1e9)
    assert b["valu_busy"] == pytest.approx(0.5)
    assert b["l1_waiting_on_l2"] == pytest.approx(0.25)
    # with this run's probe rate the peak follows the live gather rate
    b2 = bench.binding_fractions(kc, 10.0, {"l2_random_gbs": 16.0 * 200e9 / 1e9})
    assert b2["l2_peak_measured"] == pytest.approx(200e9 * 128 / 1e9)


def test_trace_overlap_sweep(tmp_path):
    rows = [("ecc::ecc_fwd_kernel(x)", 1, 0, 100), ("ecc::ecc_adj_kernel(x)", 2, 50, 150),
            ("ecc::reduce_cost_kernel(x)", 1, 200, 210), ("ecc::sino_radon_kernel(x)", 3, 0, 1000),
            ("at::native::copy(x)", 2, 0, 1000)]
    p = tmp_path / "t.csv"
    with open(p, "w") as fh:
        fh.write("Kernel_Name,Stream_Id,Queue_Id,Start_Timestamp,End_Timestamp\n")
        for n, s, t0, t1 in rows:
            fh.write(f'"{n}",{s},0,{t0},{t1}\n')
    r = bench.trace_overlap(str(p))
    assert r["kernels"] == 3  # engine evaluation kernels only
    assert r["busy_ms"] == pytest.approx(160e-6)
    assert r["two_or_more_queues_ms"] == pytest.approx(50e-6)
    assert r["max_queues_at_once"] == 2


def test_host_cpu_model_is_a_name():
    assert isinstance(bench.host_cpu_model(), str) and bench.host_cpu_model()
