"""Host-side pieces of bench.py that need no GPU: the refusal of several GPUs,
the error statistics of the error report, and the traffic guard that drops
counter figures once the kernel's sources change."""
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_relative_error_and_its_summary():
    rel = bench._rel([1.0, 2.0, 0.0], [1.0, 1.0, 0.0])
    assert rel.tolist() == [0.0, 1.0, 0.0]
    st = bench._err_stats(np.array([1e-7, 3e-6]), 1e-5, poses=2)
    assert st["results"] == 2 and st["max_rel"] == 3e-6 and st["within_bar"] and st["poses"] == 2


def test_traffic_is_dropped_when_sources_change(monkeypatch):
    monkeypatch.setitem(bench.TRAFFIC, "sources_sha256", "0" * 64)
    assert bench.measured_traffic() is None


def test_slot_accounting_is_the_documented_one():
    assert bench.SLOTS_PER_PAIR == 13.5
    assert bench.PAIR_ISSUE_SLOTS == 12
    assert abs(bench.ALU_PEAK_TSLOT - 39.3216) < 1e-9
    assert bench.SUR_FLOP_PER_POSE == 73204224


def test_matrix_core_work_counts_the_kernel_loop():
    """The closed form of unit_mfma_macs against a walk over the kernel's
    loop: sets of four block offsets t0 = 4 g, steps q < ceil((nb - t0) / 4),
    two products per offset whose first row 16 (t0 + u) + 64 q lies in the
    beam."""
    def walk(n):
        nb = (n + 15) // 16
        cnt = 0
        for g in range((nb + 3) // 4):
            t0 = 4 * g
            for q in range((nb - t0 + 3) // 4):
                for u in range(4):
                    if 16 * (t0 + u) + 64 * q < n:
                        cnt += 2
        return cnt * 1024
    lens = [1, 15, 16, 17, 63, 64, 65, 127, 128, 129, 300, 511, 512, 513, 1999, 2000]
    assert bench.unit_mfma_macs(lens) == float(sum(walk(n) for n in lens))
    assert bench.unit_mfma_macs([]) == 0.0
    # every pair is covered: at least n^2 multiply-adds
    assert all(bench.unit_mfma_macs([n]) >= n * n for n in lens)
    assert abs(bench.MFMA_F32_MAC_PEAK - 7.86432e13) < 1e6


def test_counter_figures_name_their_profiles_and_go_stale(monkeypatch):
    """Each committed counter figure names a profile summary that exists, and
    the figures are withheld once the library's sources differ from the ones
    they were taken on."""
    for name, d in bench.COUNTER_PROFILES["paths"].items():
        assert os.path.exists(os.path.join(ROOT, d["profile"])), name
        assert d["bound"] in ("alu", "mfma", "hbm")
    monkeypatch.setitem(bench.COUNTER_PROFILES, "sources_sha256", "0" * 64)
    assert bench.counter_profiles()["stale"] is True
