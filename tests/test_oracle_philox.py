"""Pins for the oracle's Philox4x32-10 (the published known-answer vectors of
the Random123 distribution, Salmon et al. SC'11) and its Gaussian sketch."""
import numpy as np
import pytest

from oracle import philox

KAT = [  # (counter, key) -> output, Philox4x32 with 10 rounds
    ((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
    ((0xFFFFFFFF,) * 4, (0xFFFFFFFF,) * 2, (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
    ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
     (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
]


@pytest.mark.parametrize("ctr,key,out", KAT)
def test_known_answers(ctr, key, out):
    got = philox.philox4x32_10([np.uint64(x) for x in ctr], [np.uint64(x) for x in key])
    assert tuple(int(x) for x in got) == out


def test_gaussian_moments():
    z = philox.gaussian_sketch(2000, 50, 1234)
    assert abs(z.mean()) < 0.01 and abs(z.std() - 1) < 0.01
    assert abs(np.mean(z ** 4) - 3.0) < 0.05          # Gaussian kurtosis
    assert not np.array_equal(z, philox.gaussian_sketch(2000, 50, 1235))
