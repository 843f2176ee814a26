"""CPU check of the histogram kernel's bin arithmetic.

The kernel computes the bin (v - offset) * num_bins / range of a U8 pixel
without a division: it takes the high 32 bits of (v - offset) * num_bins *
m with m = ceil(2^32 / range) (m = 0 when range = 1, where every counted
pixel is in bin 0).  This test restates that formula and checks it against
integer division for every range 1..256, every bin count up to the range and
every in-range value, so the device formula is exact wherever it is used."""


def _m(rng):
    return 0 if rng == 1 else -(-(1 << 32) // rng)


def test_reciprocal_fits_32_bits():
    assert all(0 <= _m(r) < (1 << 32) for r in range(1, 257))


def test_multiply_high_equals_integer_division_everywhere():
    for rng in range(1, 257):
        m = _m(rng)
        for nb in range(1, rng + 1):
            for x in range(rng):
                n = x * nb
                assert (n * m) >> 32 == n // rng, (rng, nb, x)
