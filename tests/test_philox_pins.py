"""Pins of the oracle's counter-based normal generator (oracle/philox.py),
the CPU side of the random x of the training triples (section 3.4, eq. 3.8).

Philox4x32-10 is pinned to the known-answer vectors published with the
generator's reference implementation (Random123, Salmon et al., SC 2011);
the Box-Muller normals to the standard normal distribution."""
import numpy as np
import pytest
from scipy import stats

from oracle import philox


@pytest.mark.parametrize("ctr,key,out", [
    ((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
    ((0xFFFFFFFF,) * 4, (0xFFFFFFFF, 0xFFFFFFFF), (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
    ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
     (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
])
def test_philox_known_answers(ctr, key, out):
    o = philox.philox4x32_10(np.array([ctr], dtype=np.uint64), key)[0]
    assert tuple(int(v) for v in o) == out


def test_normals_are_standard_and_independent():
    z = philox.normals(seed=7, index=3, npts=1 << 17)
    for part in (z.real, z.imag):
        assert abs(part.mean()) < 5 / np.sqrt(part.size)
        assert abs(part.var() - 1) < 5 * np.sqrt(2 / part.size)
        assert stats.kstest(part, "norm").pvalue > 1e-3
    assert abs(np.corrcoef(z.real, z.imag)[0, 1]) < 5 / np.sqrt(z.size)


def test_counter_layout_prefix_and_sample_streams():
    a = philox.normals(seed=11, index=5, npts=1000)
    b = philox.normals(seed=11, index=5, npts=300)
    np.testing.assert_array_equal(a[:300], b)      # point p depends on p only
    c = philox.normals(seed=11, index=6, npts=300)
    d = philox.normals(seed=12, index=5, npts=300)
    big = philox.normals(seed=11, index=5 + (1 << 32), npts=300)  # high index word
    for other in (c, d, big):
        assert np.abs(other - b).min() > 0 and abs(np.corrcoef(other.real, b.real)[0, 1]) < 0.2


def test_box_muller_extremes():
    """u1 = 2^-32 (word a = 0) gives the largest radius sqrt(64 ln 2); word a
    = 2^32 - 1 gives u1 = 1 and a zero sample."""
    # search the first points of one sample for the two extremes' neighbours:
    # the radius never exceeds the bound and never is negative or NaN
    z = philox.normals(seed=1, index=0, npts=1 << 16)
    assert np.all(np.isfinite(z))
    assert np.abs(z).max() <= np.sqrt(64 * np.log(2)) + 1e-12
