"""Measurement support on the GPU: the streaming read and write calibrations return rates
within what the part can physically do (above 0.5 TB/s, below the 8 TB/s HBM peak plus a
margin for a cache-resident tail), with the best time no larger than the mean."""
import pytest

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("kind", ["read", "write"])
def test_streaming_calibration_rates(bt, kind):
    fn = bt.btoep_read_bandwidth if kind == "read" else bt.btoep_write_bandwidth
    print("case calibration", kind, flush=True)
    res = fn(2 << 30, reps=2)
    assert 500.0 < res["mean_GBs"] <= res["best_GBs"] < 10000.0, res
    assert res["best_ms"] > 0.0
