"""Throughput probes of the roofline denominators (dmc_probe) on the device: they run, time themselves and
land in the range the chip's unit counts allow."""
import pytest

import paper_2403_18840_amd as dmc

pytestmark = pytest.mark.gpu

CUS, CLOCK = 256, 2.4e9


def test_probes_land_within_the_chips_unit_counts():
    ms, ops = dmc.probe(0, 2048)
    assert ms > 0 and ops > 0
    tflops = 2 * ops / (ms * 1e-3) / 1e12
    # 256 CUs x 64 FMA lanes x 2 FLOP x 2.4 GHz = 78.6 TFLOP/s unpacked; clocks may sit below 2.4 GHz
    assert 30.0 < tflops < 80.0, tflops
    for kind in (1, 2):
        ms, ops = dmc.probe(kind, 512)
        per_cu_clk = ops / (ms * 1e-3) / (CUS * CLOCK)
        assert 4.0 < per_cu_clk <= 64.0, (kind, per_cu_clk)
    ms, nbytes = dmc.probe(3, 1 << 28)
    assert nbytes == 2 * (1 << 28)
    tbs = nbytes / (ms * 1e-3) / 1e12
    assert 1.0 < tbs < 8.5, tbs
    with pytest.raises(dmc.DmcError):
        dmc.probe(4, 10)
    with pytest.raises(dmc.DmcError):
        dmc.probe(3, 17)
