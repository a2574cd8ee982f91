"""Pins of the oracle's Gaussian generator (the G of eq. power, Section 3).

The integer stream is pinned to numpy's Philox bit generator (the same
Philox4x64-10 of Salmon et al., SC'11); the Gaussian transform is pinned by
Box-Muller's identities on that stream and by distribution tests.
"""
import math

import numpy as np
import pytest
from scipy import stats

MASK = (1 << 64) - 1


def numpy_block(seed, stream, block):
    # numpy's Philox increments its 256-bit counter before each 4-word block,
    # so counter (block - 1, stream, 0, 0) yields the block at counter (block, stream, 0, 0).
    # Keys and counters go in as uint64 arrays: a Python list passes through float64.
    assert block >= 1
    bg = np.random.Philox(key=np.array([seed, 0], dtype=np.uint64),
                          counter=np.array([block - 1, stream, 0, 0], dtype=np.uint64))
    return bg.random_raw(4)


@pytest.mark.parametrize("seed", [0, 1, 1812, 2**63 + 5, MASK])
@pytest.mark.parametrize("stream", [0, 2, 3, 2**31 + 7])
@pytest.mark.parametrize("block", [1, 2, 3, 1000, 2**40 + 3])
def test_philox_matches_numpy(orc, seed, stream, block):
    got = orc.philox4x64_10([block, stream, 0, 0], [seed, 0])
    np.testing.assert_array_equal(got, numpy_block(seed, stream, block))


def test_philox_full_counter_and_key(orc):
    # all four counter words and both key words take part
    ctr = [0x243F6A8885A308D3 % (2**63), 0x13198A2E03707344, 0xA4093822299F31D0, 0x082EFA98EC4E6C89]
    key = [0x452821E638D01377, 0xBE5466CF34E90C6C]
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64),
                          counter=np.array([ctr[0] - 1] + ctr[1:], dtype=np.uint64))
    np.testing.assert_array_equal(orc.philox4x64_10(ctr, key), bg.random_raw(4))


def _unit(w):
    return ((np.asarray(w, dtype=np.uint64) >> np.uint64(11)).astype(np.float64) + 0.5) * 2.0**-53


@pytest.mark.parametrize("seed", [3, 1812])
def test_box_muller_identities(orc, seed):
    """For each pair, z_a^2 + z_b^2 = -2 ln u_a and atan2(z_b, z_a) = 2 pi u_b (mod 2 pi)."""
    rows, cols = 7, 9  # 63 values: 15 full blocks + one partial block
    G = orc.gaussian(rows, cols, seed, stream_id=2)
    flat = G.reshape(-1, order="F")
    for b in range(1, (rows * cols + 3) // 4):
        w = numpy_block(seed, 2, b)
        u = _unit(w)
        for p in range(2):
            l = 4 * b + 2 * p
            if l + 1 >= flat.size:
                continue
            za, zb = flat[l], flat[l + 1]
            assert za * za + zb * zb == pytest.approx(-2.0 * math.log(u[2 * p]), rel=1e-13)
            ang = math.atan2(zb, za) % (2 * math.pi)
            d = abs(ang - 2 * math.pi * u[2 * p + 1])
            assert min(d, 2 * math.pi - d) < 1e-12


def test_gaussian_layout_is_linear_column_major(orc):
    """Element (i,j) is number i + j*rows of one stream, whatever the shape."""
    G = orc.gaussian(13, 11, 1812, 2)
    flat = orc.gaussian(1, 13 * 11, 1812, 2).reshape(-1)
    np.testing.assert_array_equal(G.reshape(-1, order="F"), flat)
    # a different stream id or seed gives a different matrix
    assert not np.array_equal(G, orc.gaussian(13, 11, 1812, 3))
    assert not np.array_equal(G, orc.gaussian(13, 11, 1813, 2))


def test_gaussian_distribution(orc):
    z = orc.gaussian(1000, 1000, 1812, 2).reshape(-1)
    assert abs(z.mean()) < 5e-3
    assert abs(z.var() - 1.0) < 5e-3
    assert abs(stats.skew(z)) < 1e-2
    assert abs(stats.kurtosis(z)) < 2e-2
    assert stats.kstest(z, "norm").pvalue > 1e-3
    # independence of the two members of a Box-Muller pair
    pairs = z[: (z.size // 2) * 2].reshape(-1, 2)
    assert abs(np.corrcoef(pairs[:, 0], pairs[:, 1])[0, 1]) < 5e-3
