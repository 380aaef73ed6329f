"""Host-side accounting of bench.py (no GPU): refactorisations charged at their true rate."""
import os
import sys

import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402


def _st(accepts, refreshes):
    return {"accepts": accepts, "refreshes": refreshes}


def test_refresh_rate_cadence():
    # 126 accepted flips per sweep, refresh every 1024: period ceil(1024/126) = 9 sweeps
    st0 = [_st(1000, 1), _st(0, 0)]
    st1 = [_st(1000 + 20 * 126, 3), _st(20 * 63, 0)]   # second chain: 63 per sweep -> period 17
    exp, act = bench.refresh_rates(st0, st1, 20, 1024)
    assert exp == pytest.approx((20 / 9 + 20 / 17) / 2)
    assert act == pytest.approx(1.0)


def test_refresh_rate_every_sweep_and_off():
    # more accepted flips per sweep than the interval: once per sweep (checked at the sweep end)
    exp, act = bench.refresh_rates([_st(0, 0)], [_st(3 * 126, 3)], 3, 64)
    assert exp == pytest.approx(1.0 * 3) and act == 3
    # refresh off, or a chain with no accepted flip: no refactorisation due
    assert bench.refresh_rates([_st(0, 0)], [_st(500, 0)], 4, 0) == (0.0, 0.0)
    assert bench.refresh_rates([_st(7, 2)], [_st(7, 2)], 4, 64) == (0.0, 0.0)


def test_more_than_one_gpu_is_refused():
    """--gpus N > 1 ends with status 2 and a message, before anything touches a GPU."""
    import subprocess
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_record_keys():
    """Counter records are keyed by workload shape and by the window of delayed updates."""
    class A:
        L, K, group, precision, chains, delay = 8, 1, 2, 64, 4096, 0
    assert bench.traffic_key(A) == "L8_K1_Z2_p64_c4096"
    A.delay = 16
    assert bench.traffic_key(A) == "L8_K1_Z2_p64_c4096_flush16"
    assert len(bench.source_digest()) == 16 and bench.source_digest() != bench.source_digest("ggf_factor.hip")
