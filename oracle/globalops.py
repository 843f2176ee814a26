"""Oracle for global operators (Table 2: reductions and histograms).

TEST INFRASTRUCTURE ONLY (see the package docstring).  A global operator
reads every pixel of an image and produces a few values, not an image.
"""
from __future__ import annotations

import numpy as np


def histogram(img: np.ndarray, num_bins: int, offset: int, rng: int) -> np.ndarray:
    """Counts of a U8 image over ``num_bins`` equal bins of [offset, offset +
    rng): a pixel v in that interval falls in bin (v - offset) * num_bins //
    rng; pixels outside it are not counted."""
    if img.dtype != np.uint8 or not 1 <= num_bins <= 256 or rng < 1 or offset < 0 or offset + rng > 256 \
            or num_bins > rng:
        raise ValueError("U8 image, 1 <= num_bins <= range, [offset, offset + range) within 0..256")
    v = img.astype(np.int64).ravel()
    inside = (v >= offset) & (v < offset + rng)
    bins = (v[inside] - offset) * num_bins // rng
    return np.bincount(bins, minlength=num_bins).astype(np.uint32)


def min_max(img: np.ndarray) -> tuple:
    """Smallest and largest pixel of a U8 or S16 image."""
    if img.dtype not in (np.uint8, np.int16) or img.size == 0:
        raise ValueError("non-empty U8 or S16 image")
    return int(img.min()), int(img.max())


def equalize_hist(img: np.ndarray) -> np.ndarray:
    """EqualizeHist (Table 2) of a U8 image: with cdf(v) the number of pixels
    <= v, cdf_min the smallest nonzero cdf value and N the pixel count, value v
    maps to round((cdf(v) - cdf_min) * 255 / (N - cdf_min)) (halves up); an
    image of one value is returned unchanged."""
    if img.dtype != np.uint8 or img.size == 0:
        raise ValueError("non-empty U8 image")
    cdf = np.cumsum(np.bincount(img.ravel(), minlength=256)).astype(np.int64)
    n = img.size
    cmin = int(cdf[cdf > 0][0])
    if n == cmin:
        return img.copy()
    num = (cdf - cmin) * 255
    lut = (2 * num + (n - cmin)) // (2 * (n - cmin))
    lut = np.clip(lut, 0, 255).astype(np.uint8)
    return lut[img]


def min_max_count(img: np.ndarray) -> tuple:
    """Smallest and largest pixel of a U8 or S16 image and how many pixels
    take each value (the counts of MinMaxLoc)."""
    mn, mx = min_max(img)
    return mn, mx, int(np.count_nonzero(img == mn)), int(np.count_nonzero(img == mx))


def min_max_loc(img: np.ndarray) -> tuple:
    """MinMaxLoc (Table 2): the extremes, their counts and the (x, y) of
    every pixel equal to each (row-major order here; any order is a valid
    answer)."""
    mn, mx, cmin, cmax = min_max_count(img)
    ys, xs = np.nonzero(img == mn)
    lmin = [(int(x), int(y)) for y, x in zip(ys, xs)]
    ys, xs = np.nonzero(img == mx)
    lmax = [(int(x), int(y)) for y, x in zip(ys, xs)]
    return mn, mx, cmin, cmax, lmin, lmax


def mean_std_dev(img: np.ndarray) -> tuple:
    """Mean and population standard deviation of a U8 image, from the exact
    integer sums S1 = sum v and S2 = sum v^2 over N pixels: mean = S1 / N,
    stddev = sqrt(S2 / N - mean^2), in double precision.  Also returns the
    sums."""
    if img.dtype != np.uint8 or img.size == 0:
        raise ValueError("non-empty U8 image")
    v = img.astype(np.int64)
    s1, s2, n = int(v.sum()), int((v * v).sum()), img.size
    mean = s1 / n
    var = s2 / n - mean * mean
    return mean, float(np.sqrt(max(var, 0.0))), s1, s2
