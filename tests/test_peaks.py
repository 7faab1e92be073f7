"""Peak probes (fsp_probe_peak): positive rates no higher than the chip's unit
counts allow, the packed 16-bit probe at about twice the 32-bit one, and the
argument checks."""
import pytest

from helpers import require_gpu
from paper_1208_3933_amd import fspbb

pytestmark = pytest.mark.gpu

CLOCK = 2.4e9
LIMITS = {fspbb.PROBE_VALU16: 256 * 4 * 16 * 2 * CLOCK, fspbb.PROBE_VALU32: 256 * 4 * 16 * CLOCK,
          fspbb.PROBE_LDS: 256 * 256 * CLOCK, fspbb.PROBE_HBM: 8.0e12}


@pytest.mark.parametrize("kind", sorted(LIMITS))
def test_probe_rates_are_physical(kind):
    require_gpu()
    rate, ms = fspbb.probe_peak(kind, 1 << 28)
    assert ms > 0.0
    assert 0.05 * LIMITS[kind] < rate <= 1.05 * LIMITS[kind], (kind, rate)


def test_packed_probe_doubles_the_lane_rate():
    require_gpu()
    r16 = max(fspbb.probe_peak(fspbb.PROBE_VALU16)[0] for _ in range(2))
    r32 = max(fspbb.probe_peak(fspbb.PROBE_VALU32)[0] for _ in range(2))
    assert 1.6 < r16 / r32 < 2.4


def test_probe_rejects_bad_arguments():
    require_gpu()
    for kind, nbytes in [(-1, 1 << 20), (4, 1 << 20), (fspbb.PROBE_HBM, 1 << 19), (fspbb.PROBE_HBM, (1 << 20) + 8)]:
        with pytest.raises(fspbb.FspError):
            fspbb.probe_peak(kind, nbytes)
