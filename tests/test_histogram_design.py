"""CPU check of the histogram kernel's bin arithmetic.

The kernel computes the bin (v - offset) * num_bins / range of a U8 pixel
without a division and on the 24-bit multiplier: y = (v - offset) * num_bins
* 256 (mod 2^32, one multiply-add v * B + D), the pixel is counted when
y < R = range * num_bins * 256, and its bin is the high 32 bits of the
48-bit product (y mod 2^24) * m with m = ceil(2^24 / range) (m = 0 when
range = 1, where every counted pixel is in bin 0).  This test restates those
steps and checks them against integer division and the interval test for
every range 1..256, every bin count up to the range and every difference
v - offset, so the device formula is exact wherever it is used."""
import numpy as np


def _m(rng):
    return 0 if rng == 1 else -(-(1 << 24) // rng)


def test_operands_fit_the_24_bit_multiplier():
    assert all(0 <= _m(r) < (1 << 24) for r in range(1, 257))
    assert (256 << 8) < (1 << 24)            # B = num_bins * 256
    assert 256 * 256 * 256 <= (1 << 24)      # R, and y below R


def test_multiply_high_equals_integer_division_everywhere():
    for rng in range(1, 257):
        m = _m(rng)
        nb = np.arange(1, rng + 1, dtype=np.uint64)[:, None]
        x = np.arange(rng, dtype=np.uint64)[None, :]
        y = x * nb * 256                       # below 2^24 inside the interval
        assert int(y.max()) < (1 << 24)
        got = ((y & 0xFFFFFF) * np.uint64(m)) >> np.uint64(32)
        assert np.array_equal(got, (x * nb) // np.uint64(rng)), rng


def test_interval_test_on_the_wrapped_product():
    d = np.arange(-255, 256, dtype=np.int64)[None, :]   # v - offset
    for rng in range(1, 257):
        nb = np.arange(1, rng + 1, dtype=np.int64)[:, None]
        y = (d * nb * 256) % (1 << 32)
        inside = (d >= 0) & (d < rng)
        assert np.array_equal(y < rng * nb * 256, np.broadcast_to(inside, y.shape)), rng
