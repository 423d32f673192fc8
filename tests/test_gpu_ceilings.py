"""Measured device ceilings (ocean_device_ceilings): positive and within the published peaks
of the part (FP64 matrix cores and FP64 vector units 78.6 TFLOP/s each, HBM 8 TB/s), with a
5% margin for the clock."""
import pytest

pytestmark = pytest.mark.gpu


def test_device_ceilings_within_published_peaks():
    import paper_1601_07728_amd as ob
    print("[ceilings] 256 MiB copy", flush=True)
    c = ob.device_ceilings(1 << 28)
    assert 5.0 < c["mfma_f64_tflops"] <= 78.6 * 1.05, c
    assert 5.0 < c["fma_f64_tflops"] <= 78.6 * 1.05, c
    assert 500.0 < c["copy_GBs"] <= 8000.0 * 1.05, c
    assert 500.0 < c["read_GBs"] <= 8000.0 * 1.05, c


def test_device_ceilings_rejects_small_copy():
    import paper_1601_07728_amd as ob
    with pytest.raises(ob.OceanError):
        ob.device_ceilings(1024)
