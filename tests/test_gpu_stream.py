"""The roofline's bandwidth reference: a plain 3-read + 1-write stream runs
and reports a rate between a tenth of the HBM peak and the peak."""
import pytest

pytestmark = pytest.mark.gpu


def test_stream_bandwidth_is_plausible():
    from paper_1808_01995_amd import _abi
    g = _abi.wf_stream_bandwidth(1 << 26, 5)
    print("stream %.1f GB/s" % g)
    assert 800.0 < g < 8000.0
    # a size that is not a multiple of 4 floats
    assert _abi.wf_stream_bandwidth((1 << 20) + 3, 2) > 0.0
