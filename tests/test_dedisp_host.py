"""Host side of the dedispersion library (no GPU): the delay table the C
library computes equals the oracle's, and bad arguments are refused."""
import numpy as np
import pytest

from oracle import dedisp_oracle as dd
from synth import filterbank as fb


def sps():
    from paper_2512_00398_amd import sps as m
    return m


@pytest.mark.parametrize("nchan,ndm,dm_max,tsamp", [(1024, 1024, 1000.0, 49.152e-6), (64, 33, 3000.0, 1e-3),
                                                   (300, 7, 57.5, 64e-6)])
def test_library_delays_equal_oracle(nchan, ndm, dm_max, tsamp):
    f, fref = fb.band(nchan)
    dms = np.linspace(0, dm_max, ndm).astype(np.float32)
    lib = sps().dedisp_delays(f, fref, tsamp, dms)
    ref = dd.delays(f, fref, tsamp, dms)
    assert lib.dtype == np.int32 and np.array_equal(lib.astype(np.int64), ref)


def test_library_delays_reject_bad_arguments():
    m = sps()
    with pytest.raises(m.SpsError):
        m.dedisp_delays([1500.0], 1450.0, 1e-4, [1.0])  # channel above the reference
    with pytest.raises(m.SpsError):
        m.dedisp_delays([1400.0], 1450.0, 0.0, [1.0])  # tsamp
    with pytest.raises(m.SpsError):
        m.dedisp_delays([1400.0], 1450.0, 1e-4, [-1.0])  # negative DM
    with pytest.raises(m.SpsError):
        m.dedisp_delays([1.0], 1450.0, 1e-9, [1e6])  # beyond int32
