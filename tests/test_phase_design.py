"""CPU check of the packed half-precision Phase arithmetic the GPU kernels use.

The kernels compute the Phase level (Table 2: atan2(gy, gx) on [0, 2 pi)
mapped to 256 levels) with half-precision operations.  This test repeats
those steps in numpy, rounding each one to half precision as the hardware
does (numpy's float16 rounds to nearest even and keeps subnormals), and
checks over every (gx, gy) in [-1023, 1023]^2 that the level is within one
of round(exact level), the tolerance the GPU parity tests apply.  It takes
no value from the oracle; the exact level comes from numpy's arctan2 in
float64.  It guards the design (constants, scalings, octant code), not the
compiled kernel, which the GPU tests compare against the oracle."""
import numpy as np

F16 = np.float16


def _rnd(x):
    return np.asarray(x, np.float64).astype(F16).astype(np.float64)


def _bits(x):
    return np.asarray(x, np.float64).astype(F16).view(np.uint16).astype(np.int64)


def _half(b):
    return np.asarray(np.asarray(b) & 0xFFFF, np.uint16).view(F16).astype(np.float64)


# constants of the kernel's phase function
MAGIC = 0x8F9C             # 2^6 / F ~ half(MAGIC - bits(F)), 16-bit wrap-around
C0, C1 = 345.0, 712.0      # 8 c0 and 64 c1, c1 = 0.273 * 128 / pi, c0 = 32 + c1
NEG = [0x00, 0xFF, 0x00, 0xFF, 0x00, 0xFF, 0x00, 0xFF]
ADD = [0x00, 0x41, 0x40, 0x81, 0x80, 0xC1, 0xC0, 0x01]


def _levels(gx, gy):
    ax, ay = np.abs(gx), np.abs(gy)
    mn, mx = np.minimum(ax, ay), np.maximum(ax, ay)
    F = _rnd(_half(mx) * 32768.0)          # mx 2^-24 (subnormal) times 2^15
    R = _half(MAGIC - _bits(F))
    E = _rnd(128.0 - F * R)
    zz = _rnd(_rnd(_half(mn) * R) * E)     # z / 8
    p = _rnd(C0 - C1 * zz)
    a = _bits(_rnd(zz * p + 1024.0)) & 0xFF
    d = (ax - ay) & 0xFFFF
    t = (gy & 0xFFFF) ^ ((gx & 0xFFFF) & 0x6000) ^ (d & 0x2000)
    o = t >> 13
    return ((a ^ np.array(NEG)[o]) + np.array(ADD)[o]) & 0xFF, a


def test_constants_are_the_rounded_coefficients():
    c1 = 0.273 * 128 / np.pi
    assert abs(C1 / 64 - c1) < 2 ** -4 and abs(C0 / 8 - (32 + c1)) < 2 ** -3
    assert _rnd(C0) == C0 and _rnd(C1) == C1
    # the estimate of 2^6 / F is within 7% for every F the kernel forms
    F = _rnd(_half(np.arange(1, 1024)) * 32768.0)
    R = _half(MAGIC - _bits(F))
    assert np.all(np.abs(R * F / 64 - 1) < 0.07)


def test_phase_levels_within_one_over_the_sobel_range():
    r = np.arange(-1023, 1024, dtype=np.int64)
    worst_alpha, worst_level = 0.0, 0
    for i0 in range(0, r.size, 256):
        gx, gy = np.meshgrid(r, r[i0:i0 + 256])
        lev, a = _levels(gx, gy)
        th = np.arctan2(gy.astype(np.float64), gx.astype(np.float64))
        th = np.where(th < 0, th + 2 * np.pi, th)
        ref = np.floor(th * 128 / np.pi + 0.5).astype(np.int64) % 256
        diff = np.abs(lev - ref) % 256
        worst_level = max(worst_level, int(np.minimum(diff, 256 - diff).max()))
        ax, ay = np.abs(gx), np.abs(gy)
        mn, mx = np.minimum(ax, ay), np.maximum(ax, ay)
        exact = np.where(mx == 0, 0.0, np.arctan2(mn, np.maximum(mx, 1)) * 128 / np.pi)
        worst_alpha = max(worst_alpha, float(np.abs(a - exact).max()))
    assert worst_alpha < 0.75
    assert worst_level <= 1


def test_octant_code_matches_the_quadrant_rules():
    # one point inside each octant and on each axis, against the level formula
    pts = [(100, 30), (30, 100), (-30, 100), (-100, 30), (-100, -30), (-30, -100), (30, -100), (100, -30),
           (50, 0), (0, 50), (-50, 0), (0, -50), (0, 0), (40, 40), (-40, -40)]
    gx = np.array([p[0] for p in pts], np.int64)
    gy = np.array([p[1] for p in pts], np.int64)
    lev, _ = _levels(gx, gy)
    th = np.mod(np.arctan2(gy, gx), 2 * np.pi) * 128 / np.pi
    ref = np.floor(th + 0.5).astype(np.int64) % 256
    assert list(ref[8:13]) == [0, 64, 128, 192, 0]
    d = np.abs(lev - ref) % 256
    assert np.all(np.minimum(d, 256 - d) <= 1)


# the variant for gradients held as half-precision bit patterns (sign and
# subnormal magnitude), which the fused edge + phase kernels form directly
ADD_SM = [0x00, 0x00, 0x00, 0xC0, 0x80, 0x00, 0x00, 0x40]


def _sign_magnitude(g):
    return ((g < 0).astype(np.int64) << 15) | np.abs(g)


def _bitop3(s0, s1, s2, tt):
    """v_bitop3_b32 on 16-bit values: bit i of tt is the result for
    (s0, s1, s2) = (i >> 2 & 1, i >> 1 & 1, i & 1)."""
    r = np.zeros_like(s0)
    for i in range(8):
        if (tt >> i) & 1:
            r |= (s0 if i & 4 else ~s0) & (s1 if i & 2 else ~s1) & (s2 if i & 1 else ~s2)
    return r & 0xFFFF


def _levels_sm(gx, gy):
    hx, hy = _sign_magnitude(gx), _sign_magnitude(gy)
    ax, ay = hx & 0x7FFF, hy & 0x7FFF
    mn, mx = np.minimum(ax, ay), np.maximum(ax, ay)
    F = _rnd(_half(mx) * 32768.0)
    R = _half(MAGIC - _bits(F))
    E = _rnd(128.0 - F * R)
    zz = _rnd(_rnd(_half(mn) * R) * E)
    p = _rnd(C0 - C1 * zz)
    d = (hx - hy) & 0xFFFF                 # |gx| - |gy| + 2^15 (s2 ^ s3)
    ps = np.where(d >> 15, -p, p)          # the sign of the factor: alpha negated
    a = _bits(_rnd(zz * ps + 1280.0)) & 0xFF
    o = _bitop3(hx, hy, d, 0x72) >> 13
    return (a + np.array(ADD_SM)[o]) & 0xFF


def test_sign_magnitude_variant_gives_the_same_levels():
    r = np.arange(-1023, 1024, dtype=np.int64)
    for i0 in range(0, r.size, 256):
        gx, gy = np.meshgrid(r, r[i0:i0 + 256])
        lev, _ = _levels(gx, gy)
        assert np.array_equal(_levels_sm(gx, gy), lev)


def test_half_precision_gradients_are_sign_magnitude_integers():
    # sums and differences of integers below 1024 in half precision, as the
    # kernels form Sobel gradients, are exact and give sign | magnitude,
    # with +0 for a zero difference
    rng = np.random.default_rng(5)
    a = rng.integers(0, 1021, 200000)
    b = rng.integers(0, 1021, 200000)
    a[:1000] = b[:1000]
    diff = _bits(_half(a) - _half(b))
    assert np.array_equal(diff, _sign_magnitude(a - b))
    u = rng.integers(-510, 511, 200000)
    v = rng.integers(-510, 511, 200000)
    s = _bits(_half(_sign_magnitude(u)) + _half(_sign_magnitude(v)))
    assert np.array_equal(s, _sign_magnitude(u + v))
