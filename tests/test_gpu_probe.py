"""The measurement probes: latency floor and HBM streaming bandwidth are
physical quantities of the device, so they must be positive and the
bandwidths below the published 8 TB/s HBM3E peak (with 5% slack for the
rounding of the timers)."""
import pytest

pytestmark = pytest.mark.gpu


def test_latency_probe():
    from paper_2605_11673_amd import stafem
    f = stafem.latency_probe()
    assert 0.1 < f["empty_kernel_us"] < 100
    assert 0 < f["dependent_load_l2_ns"] <= f["dependent_load_256MB_ns"] * 1.5
    assert 0 < f["dependent_atomic_ns"] < 1e5


def test_bandwidth_probe():
    from paper_2605_11673_amd import stafem
    b = stafem.bandwidth_probe()
    for k in ("read_GBs", "write_GBs", "copy_GBs"):
        assert 100.0 < b[k] < 8000.0 * 1.05, (k, b[k])
