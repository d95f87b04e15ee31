"""The bandwidth probes behind the bench's measured peaks: both run and land
in the range the hardware allows (MI355X: 8 TB/s HBM, 256 CUs of LDS)."""
import pytest

from paper_1909_10286_amd import bl

pytestmark = pytest.mark.gpu


def test_measured_peaks_are_plausible(ctx):
    hbm, lds = ctx.measure_peaks()
    assert 1000.0 < hbm < 8000.0, hbm          # copy: read + written bytes, below the HBM peak
    assert 20000.0 < lds < 400000.0, lds       # 16-byte LDS reads on every CU
    assert lds > 5 * hbm
