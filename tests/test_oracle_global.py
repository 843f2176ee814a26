"""Pins of the global-operator oracle against numpy's own histogram, mean
and standard deviation, and brute force on tiny images."""
import numpy as np
import pytest

from oracle import globalops as G

RNG = np.random.default_rng(9)
IMG = RNG.integers(0, 256, (37, 53), dtype=np.uint8)


@pytest.mark.parametrize("bins,offset,rng", [(256, 0, 256), (16, 0, 256), (10, 20, 200), (1, 0, 256), (7, 100, 21)])
def test_histogram_matches_numpy_histogram(bins, offset, rng):
    # numpy's half-open bins on the edges offset + k * rng / bins (exact for these pairs)
    edges = offset + np.arange(bins + 1) * (rng / bins)
    want, _ = np.histogram(IMG, bins=edges)
    last = IMG == offset + rng  # np.histogram closes the last bin; the OpenVX interval is half-open
    want[-1] -= last.sum() if edges[-1] == offset + rng else 0
    assert np.array_equal(G.histogram(IMG, bins, offset, rng), want)
    assert G.histogram(IMG, bins, offset, rng).sum() == ((IMG >= offset) & (IMG < offset + rng)).sum()


def test_histogram_brute_force_uneven_bins():
    img = np.arange(256, dtype=np.uint8).reshape(16, 16)
    got = G.histogram(img, 3, 10, 10)  # bins of width 10/3: 10..13, 14..16, 17..19
    assert got.tolist() == [4, 3, 3]


def test_min_max_brute_force():
    for dt, lo, hi in ((np.uint8, 0, 256), (np.int16, -32768, 32768)):
        img = RNG.integers(lo, hi, (5, 7)).astype(dt)
        flat = [int(x) for x in img.ravel()]
        m, M = flat[0], flat[0]
        for x in flat:
            m, M = (x if x < m else m), (x if x > M else M)
        assert G.min_max(img) == (m, M)


def test_min_max_count_brute_force():
    img = np.array([[3, 9, 3], [9, 1, 9]], np.uint8)
    assert G.min_max_count(img) == (1, 9, 1, 3)
    const = np.full((4, 4), -5, np.int16)
    assert G.min_max_count(const) == (-5, -5, 16, 16)
    for dt, lo, hi in ((np.uint8, 0, 4), (np.int16, -3, 3)):
        img = RNG.integers(lo, hi, (6, 5)).astype(dt)
        flat = [int(x) for x in img.ravel()]
        m, M = min(flat), max(flat)
        assert G.min_max_count(img) == (m, M, sum(1 for x in flat if x == m), sum(1 for x in flat if x == M))


def test_equalize_hist_worked_example_and_properties():
    # four values with counts 1, 2, 3, 2 (N = 8): cdf 1, 3, 6, 8, cdf_min 1, so the levels are
    # round(0), round(2 * 255 / 7) = round(72.86), round(5 * 255 / 7) = round(182.14), 255
    img = np.array([[10, 20, 20, 30], [30, 30, 40, 40]], np.uint8)
    assert G.equalize_hist(img).tolist() == [[0, 73, 73, 182], [182, 182, 255, 255]]
    # a half rounds up: N - cdf_min = 2, values 0 / 127.5 / 255
    assert G.equalize_hist(np.array([[5, 6, 7]], np.uint8)).tolist() == [[0, 128, 255]]
    const = np.full((3, 3), 42, np.uint8)
    assert np.array_equal(G.equalize_hist(const), const)
    out = G.equalize_hist(IMG)
    order = np.argsort(IMG.ravel(), kind="stable")
    assert np.all(np.diff(out.ravel()[order].astype(int)) >= 0)  # monotone in the input value
    assert out.min() == 0 and out.max() == 255


def test_min_max_loc_brute_force():
    img = np.array([[3, 9, 3], [9, 1, 9]], np.uint8)
    assert G.min_max_loc(img) == (1, 9, 1, 3, [(1, 1)], [(1, 0), (0, 1), (2, 1)])
    img = RNG.integers(0, 3, (4, 6)).astype(np.int16)
    mn, mx, cmin, cmax, lmin, lmax = G.min_max_loc(img)
    assert sorted(lmin) == sorted((x, y) for y in range(4) for x in range(6) if img[y, x] == mn)
    assert sorted(lmax) == sorted((x, y) for y in range(4) for x in range(6) if img[y, x] == mx)
    assert len(lmin) == cmin and len(lmax) == cmax


def test_mean_std_dev_matches_numpy():
    mean, std, s1, s2 = G.mean_std_dev(IMG)
    assert mean == pytest.approx(float(np.mean(IMG, dtype=np.float64)), rel=1e-15)
    assert std == pytest.approx(float(np.std(IMG, dtype=np.float64)), rel=1e-12)
    const = np.full((3, 4), 77, np.uint8)
    assert G.mean_std_dev(const)[:2] == (77.0, 0.0)
    two = np.array([[0, 255]], np.uint8)
    assert G.mean_std_dev(two)[:2] == (127.5, 127.5)
