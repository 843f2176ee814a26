"""Pins of the CPU reference against facts that do not come from the reference
itself: library routines (scipy.ndimage) that implement the same textbook
operation, closed forms, invariants, exhaustive checks and hand-worked
examples.  Each test is chosen so that a plausible slip in the reference (a
wrong weight, sign, index, border rule or rounding) fails it."""
import math
import os

import numpy as np
import pytest
import scipy.ndimage as nd

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
SIZES = [(1, 1), (2, 3), (3, 2), (7, 5), (17, 13), (33, 4)]
BORDERS = [("replicate", 0), ("constant", 0), ("constant", 77), ("constant", 255), ("mirror", 0), ("repeat", 0)]


def _nd_mode(border, c):
    if border == "mirror":
        return "mirror", 0  # scipy's reflect-101 extension
    if border == "repeat":
        return "wrap", 0  # scipy's periodic extension
    return ("nearest", 0) if border == "replicate" else ("constant", c)


def _corr(img, k, border, c):
    mode, cval = _nd_mode(border, c)
    return nd.correlate(img.astype(np.int64), np.asarray(k, np.int64), mode=mode, cval=cval)


def _read_golden(name):
    blocks, cur = {}, None
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line[0].isalpha():
                cur = blocks.setdefault(line, [])
            else:
                cur.append([int(v) for v in line.split()])
    return {k: np.array(v) for k, v in blocks.items()}


# ---- local operators vs a library correlation ---------------------------

@pytest.mark.parametrize("w,h", SIZES)
@pytest.mark.parametrize("border,c", BORDERS)
def test_gaussian_box_vs_scipy(w, h, border, c):
    img = synth.uniform_u8(w, h, seed=w * 131 + h)
    g3 = np.outer([1, 2, 1], [1, 2, 1])
    g5 = np.outer([1, 4, 6, 4, 1], [1, 4, 6, 4, 1])
    assert np.array_equal(oracle.gaussian3x3(img, border, c), _corr(img, g3, border, c) >> 4)
    assert np.array_equal(oracle.gaussian5x5(img, border, c), _corr(img, g5, border, c) >> 8)
    assert np.array_equal(oracle.box3x3(img, border, c), _corr(img, np.ones((3, 3)), border, c) // 9)


@pytest.mark.parametrize("w,h", SIZES)
@pytest.mark.parametrize("border,c", BORDERS)
def test_dilate_erode_median_vs_scipy(w, h, border, c):
    """Grey dilation, erosion and the median filter of scipy.ndimage over the
    3x3 window, with the same border extension."""
    img = synth.uniform_u8(w, h, seed=w * 7 + h)
    mode, cval = _nd_mode(border, c)
    kw = dict(size=(3, 3), mode=mode, cval=cval)
    assert np.array_equal(oracle.dilate3x3(img, border, c), nd.grey_dilation(img, **kw))
    assert np.array_equal(oracle.erode3x3(img, border, c), nd.grey_erosion(img, **kw))
    assert np.array_equal(oracle.median3x3(img, border, c), nd.median_filter(img, **kw))


PATTERNS = {"box3": np.ones((3, 3)), "cross3": np.array([[0, 1, 0], [1, 1, 1], [0, 1, 0]]),
            "disk5": np.array([[0, 1, 1, 1, 0]] + [[1] * 5] * 3 + [[0, 1, 1, 1, 0]]),
            "custom5x3": np.array([[1, 0, 0, 1, 1], [0, 1, 1, 0, 1], [1, 1, 0, 0, 0]]),
            "pair1x3": np.array([[1, 0, 1]])}


@pytest.mark.parametrize("pattern", sorted(PATTERNS))
@pytest.mark.parametrize("border,c", BORDERS)
def test_nonlinear_vs_scipy(pattern, border, c):
    """NonLinearFilter over a mask against scipy.ndimage's rank filters with
    the same footprint (median: rank n // 2, which scipy's median filter uses)."""
    img = synth.uniform_u8(23, 17, seed=len(pattern) + c)
    m = PATTERNS[pattern]
    mode, cval = _nd_mode(border, c)
    kw = dict(footprint=m != 0, mode=mode, cval=cval)
    assert np.array_equal(oracle.nonlinear(img, m, "min", border, c), nd.minimum_filter(img, **kw))
    assert np.array_equal(oracle.nonlinear(img, m, "max", border, c), nd.maximum_filter(img, **kw))
    assert np.array_equal(oracle.nonlinear(img, m, "median", border, c), nd.median_filter(img, **kw))
    if pattern == "box3":
        assert np.array_equal(oracle.nonlinear(img, m, "median", border, c), oracle.median3x3(img, border, c))


@pytest.mark.parametrize("win", [3, 5])
@pytest.mark.parametrize("border,c", [("constant", -32768), ("replicate", 0), ("mirror", 0), ("repeat", 0)])
def test_nonmax_distinct_values_equals_strict_local_maxima(win, border, c):
    """With all values distinct (a permutation in S16) and none equal to the
    constant border, a pixel is kept exactly where it is the maximum of its
    window (scipy's maximum filter), except where the border mode maps a
    window position before it in raster order onto the pixel itself: that
    copy ties, and a tie before the pixel suppresses it.  Replicate does so on
    row 0 and column 0; reflect-101 on row 1 and column 1 for a 5x5 window."""
    rng = np.random.default_rng(win)
    h, w = 29, 31
    img = (rng.permutation(h * w) - 400).astype(np.int16).reshape(h, w)
    mode, cval = _nd_mode(border, c)
    keep = img == nd.maximum_filter(img, size=win, mode=mode, cval=cval)
    yy, xx = np.mgrid[0:h, 0:w]
    if border == "replicate":
        keep &= (yy != 0) & (xx != 0)
    if border == "mirror" and win == 5:
        keep &= (yy != 1) & (xx != 1)
    assert np.array_equal(oracle.nonmax(img, win, border, c), np.where(keep, img, np.int16(-32768)))


def test_nonmax_plateaus_keep_their_first_pixel():
    """A plateau of equal maxima keeps only its first pixel in raster order;
    a lone peak survives, everything else takes the format's minimum."""
    img = np.zeros((7, 9), np.uint8)
    img[2, 3:6] = 50       # a horizontal plateau: keep (2, 3)
    img[4:6, 1] = 80       # a vertical plateau: keep (4, 1)
    img[5, 7] = 90         # a lone peak
    got = oracle.nonmax(img, 3, "constant", 0)
    kept = np.argwhere(got != 0).tolist()
    assert kept == [[2, 3], [4, 1], [5, 7]]
    assert got[2, 3] == 50 and got[4, 1] == 80 and got[5, 7] == 90
    const = np.full((4, 5), 9, np.uint8)
    assert np.argwhere(oracle.nonmax(const, 5, "constant", 0) != 0).tolist() == [[0, 0]]
    s = np.full((3, 3), -5, np.int16)
    assert oracle.nonmax(s, 3, "constant", -32768)[0, 0] == -5 and (oracle.nonmax(s, 3, "constant", -32768) == -32768).sum() == 8


def test_dilate_erode_median_brute_force_and_order():
    """Brute force over explicit windows on a small image, and the order
    erode <= median <= dilate with equality on a constant image."""
    rng = np.random.default_rng(3)
    img = rng.integers(0, 256, size=(6, 7)).astype(np.uint8)
    pad = np.pad(img.astype(np.int64), 1, mode="edge")
    win = np.stack([pad[j:j + 6, i:i + 7] for j in range(3) for i in range(3)])
    assert np.array_equal(oracle.dilate3x3(img), win.max(0))
    assert np.array_equal(oracle.erode3x3(img), win.min(0))
    assert np.array_equal(oracle.median3x3(img), np.sort(win, axis=0)[4])
    big = synth.uniform_u8(40, 30, seed=5)
    e, m, d = oracle.erode3x3(big), oracle.median3x3(big), oracle.dilate3x3(big)
    assert np.all(e <= m) and np.all(m <= d) and np.all(e <= big) and np.all(big <= d)
    const = np.full((5, 9), 77, np.uint8)
    for f in (oracle.erode3x3, oracle.median3x3, oracle.dilate3x3):
        assert np.array_equal(f(const, "constant", 77), const)
    # a lone bright pixel grows to a 3x3 square under dilation, vanishes under
    # erosion and the median
    dot = np.zeros((7, 7), np.uint8)
    dot[3, 3] = 200
    assert oracle.dilate3x3(dot)[2:5, 2:5].min() == 200 and oracle.dilate3x3(dot).sum() == 9 * 200
    assert oracle.erode3x3(dot).max() == 0 and oracle.median3x3(dot).max() == 0


@pytest.mark.parametrize("w,h", SIZES)
@pytest.mark.parametrize("border,c", BORDERS)
def test_sobel_vs_scipy_sobel(w, h, border, c):
    img = synth.uniform_u8(w, h, seed=w * 7 + h)
    mode, cval = _nd_mode(border, c)
    gx, gy = oracle.sobel3x3(img, border, c)
    if border == "replicate":
        # scipy's sobel: central difference along `axis`, (1 2 1) smoothing
        # across it.  Its two separable passes pad each pass on its own, which
        # equals the 2-D window only for the nearest-pixel border.
        assert np.array_equal(gx, nd.sobel(img.astype(np.int64), axis=1, mode=mode))
        assert np.array_equal(gy, nd.sobel(img.astype(np.int64), axis=0, mode=mode))
    kx = np.outer([1, 2, 1], [-1, 0, 1])
    assert np.array_equal(gx, _corr(img, kx, border, c))
    assert np.array_equal(gy, _corr(img, kx.T, border, c))


def test_golden_gaussian_hand_worked():
    g = _read_golden("gaussian3x3_hand.txt")
    assert np.array_equal(oracle.gaussian3x3(g["A input"].astype(np.uint8), "replicate"), g["A output"])
    assert np.array_equal(oracle.gaussian3x3(g["B input"].astype(np.uint8), "constant", 0), g["B output"])


# ---- invariants and closed forms ----------------------------------------

@pytest.mark.parametrize("v", [0, 1, 128, 255])
def test_constant_image_invariants(v):
    img = np.full((9, 11), v, np.uint8)
    for f in (oracle.gaussian3x3, oracle.gaussian5x5, oracle.box3x3):
        assert np.all(f(img, "replicate") == v)
        out0 = f(img, "constant", 0)
        r = 2 if f is oracle.gaussian5x5 else 1
        assert np.all(out0[r:-r, r:-r] == v)
    gx, gy = oracle.sobel3x3(img, "replicate")
    assert not gx.any() and not gy.any()
    gx, gy = oracle.sobel3x3(img, "constant", 0)
    assert not gx[1:-1, 1:-1].any() and not gy[1:-1, 1:-1].any()
    if v:  # the CONSTANT(0) frame differs from the image: the invariant must break there
        assert gx[:, 0].min() > 0 and gy[0, :].min() > 0


@pytest.mark.parametrize("a,b,c", [(1, 0, 3), (0, 1, 5), (2, 3, 10), (-3, 2, 120), (5, -4, 100)])
def test_ramp_closed_forms(a, b, c):
    h, w = 12, 14
    yy, xx = np.mgrid[0:h, 0:w]
    img = (a * xx + b * yy + c).astype(np.int64)
    assert img.min() >= 0 and img.max() <= 255
    img = img.astype(np.uint8)
    for f in (oracle.gaussian3x3, oracle.gaussian5x5):
        r = 1 if f is oracle.gaussian3x3 else 2
        assert np.array_equal(f(img, "replicate")[r:-r, r:-r], img[r:-r, r:-r])
    gx, gy = oracle.sobel3x3(img, "replicate")
    assert np.all(gx[1:-1, 1:-1] == 8 * a) and np.all(gy[1:-1, 1:-1] == 8 * b)
    # REPLICATE edge columns/rows: one side of the difference is the pixel itself
    assert np.all(gx[1:-1, 0] == 4 * a) and np.all(gx[1:-1, -1] == 4 * a)
    assert np.all(gy[0, 1:-1] == 4 * b) and np.all(gy[-1, 1:-1] == 4 * b)
    # Gaussian then Sobel of a ramp: still the ramp's gradient in the interior
    gx2, gy2 = oracle.sobel3x3(oracle.gaussian3x3(img, "replicate"), "replicate")
    assert np.all(gx2[2:-2, 2:-2] == 8 * a) and np.all(gy2[2:-2, 2:-2] == 8 * b)
    m = oracle.magnitude(gx, gy)
    assert np.all(m[1:-1, 1:-1] == round(8 * math.hypot(a, b)))


# ---- point operators ------------------------------------------------------

def test_magnitude_exhaustive_sobel_range():
    r = np.arange(-1020, 1021, dtype=np.int16)
    gx, gy = np.meshgrid(r, r)
    m = oracle.magnitude(gx, gy)
    s = gx.astype(np.float64) ** 2 + gy.astype(np.float64) ** 2
    # nearest tie of sqrt(s) for integer s <= 2.1e6 is > 2.7e-6 away from x.5,
    # far beyond the double rounding error, so this is the exact rounding
    assert np.array_equal(m, np.floor(np.sqrt(s) + 0.5).astype(np.int16))


def test_magnitude_full_s16_range_and_saturation():
    a = synth.uniform_s16(512, 64, seed=3)
    b = synth.uniform_s16(512, 64, seed=4)
    m = oracle.magnitude(a, b).astype(np.int64)
    s = a.astype(np.float64) ** 2 + b.astype(np.float64) ** 2
    assert np.array_equal(m, np.minimum(np.floor(np.sqrt(s) + 0.5), 32767).astype(np.int64))
    ex = np.array([[-32768, 3, 0, 32767]], np.int16)
    ey = np.array([[-32768, 4, 0, 0]], np.int16)
    assert oracle.magnitude(ex, ey).tolist() == [[32767, 5, 0, 32767]]


def test_threshold_of_magnitude_rewrite():
    # round(sqrt(s)) > t  <=>  s > t*t + t for integer t >= 0: the test of the
    # strength reduction the fused edge kernel relies on (exhaustive).
    r = np.arange(-1020, 1021, dtype=np.int16)
    gx, gy = np.meshgrid(r, r)
    s = gx.astype(np.int64) ** 2 + gy.astype(np.int64) ** 2
    m = oracle.magnitude(gx, gy)
    for t in (0, 1, 2, 99, 100, 101, 1000, 1442, 1443):
        assert np.array_equal(oracle.threshold(m, t) == 255, s > t * t + t)


def test_phase_exact_points():
    pts = {(1, 0): 0, (1, 1): 32, (0, 1): 64, (-1, 1): 96, (-1, 0): 128, (-1, -1): 160, (0, -1): 192,
           (1, -1): 224, (0, 0): 0, (1000, -1): 0, (5, 0): 0}
    gx = np.array([[p[0] for p in pts]], np.int16)
    gy = np.array([[p[1] for p in pts]], np.int16)
    assert oracle.phase(gx, gy).tolist() == [list(pts.values())]


def test_phase_rotation_and_mirror():
    rng = np.random.default_rng(5)
    gx = rng.integers(-1020, 1021, size=(64, 64)).astype(np.int16)
    gy = rng.integers(-1020, 1021, size=(64, 64)).astype(np.int16)
    p = oracle.phase(gx, gy).astype(int)
    p90 = oracle.phase(-gy, gx).astype(int)  # rotate the vector by +90 degrees
    pm = oracle.phase(gx, -gy).astype(int)  # mirror about the x axis
    nz = (gx != 0) | (gy != 0)

    def circ(a, b):
        d = np.abs(a - b) % 256
        return np.minimum(d, 256 - d)

    assert circ(p90, (p + 64) % 256)[nz].max() <= 1
    assert (circ(p90, (p + 64) % 256)[nz] == 0).mean() > 0.999
    assert circ(pm, (256 - p) % 256)[nz].max() <= 1
    # quadrant of the phase follows the signs of the gradient
    q = p // 64
    sel = (gx > 0) & (gy > 0) & (p % 64 != 0)
    assert np.all(q[sel] == 0)
    sel = (gx < 0) & (gy < 0) & (p % 64 != 0)
    assert np.all(q[sel] == 2)


def test_threshold_strict_and_values():
    img = np.array([[99, 100, 101, 255, 0]], np.uint8)
    assert oracle.threshold(img, 100).tolist() == [[0, 0, 255, 255, 0]]
    assert oracle.threshold(img, 100, 7, 9).tolist() == [[9, 9, 7, 7, 9]]
    s16 = np.array([[-5, 0, 100, 101]], np.int16)
    assert oracle.threshold(s16, 100).tolist() == [[0, 0, 0, 255]]
    f = np.array([[1e6, 1e6 + 1e-3, -1e7]])
    assert oracle.threshold(f, 1e6).tolist() == [[0, 255, 0]]


def test_add_policies():
    a = np.array([[250, 10, 0]], np.uint8)
    b = np.array([[10, 20, 0]], np.uint8)
    assert oracle.add(a, b, "u8", "saturate").tolist() == [[255, 30, 0]]
    assert oracle.add(a, b, "u8", "wrap").tolist() == [[4, 30, 0]]
    c = np.array([[32767, -32768, -5]], np.int16)
    d = np.array([[1, -1, 3]], np.int16)
    assert oracle.add(c, d, "s16", "saturate").tolist() == [[32767, -32768, -2]]
    assert oracle.add(c, d, "s16", "wrap").tolist() == [[-32768, 32767, -2]]
    assert oracle.add(a, d.astype(np.int16), "s16", "saturate").tolist() == [[251, 9, 3]]


def test_channel_extract_positions():
    f = synth.uyvy_image(6, 3, seed=1)
    y = oracle.channel_extract_y(f)
    assert np.array_equal(y, f[:, 1::2])
    assert np.array_equal(y, synth.edge_image(6, 3, seed=1))


@pytest.mark.parametrize("border,c", BORDERS[:3])
def test_convolve_vs_scipy(border, c):
    img = synth.uniform_u8(13, 9, seed=11)
    mask = np.array([[1, -2, 3], [0, 4, -5], [6, 0, -1]], np.int16)  # asymmetric: pins the 180 degree rotation
    mode, cval = _nd_mode(border, c)
    s = nd.convolve(img.astype(np.int64), mask.astype(np.int64), mode=mode, cval=cval)
    for scale in (1, 2, 16):
        q = np.trunc(s / scale).astype(np.int64)  # toward zero
        assert np.array_equal(oracle.convolve(img, mask, scale, "s16", border, c), np.clip(q, -32768, 32767))
        assert np.array_equal(oracle.convolve(img, mask, scale, "u8", border, c), np.clip(q, 0, 255))
    lap = np.array([[0, 1, 0], [1, -4, 1], [0, 1, 0]], np.int16)  # the Laplacian test mask of Section 6
    ramp = (np.arange(9)[:, None] * 3 + np.arange(13)[None, :] * 2).astype(np.uint8)
    assert not oracle.convolve(ramp, lap, 1, "s16", "replicate")[1:-1, 1:-1].any()
    m5 = np.arange(25, dtype=np.int16).reshape(5, 5) - 12
    s5 = nd.convolve(img.astype(np.int64), m5.astype(np.int64), mode=mode, cval=cval)
    assert np.array_equal(oracle.convolve(img, m5, 4, "s16", border, c), np.trunc(s5 / 4).astype(np.int64))


# ---- the corner (Harris) response in double precision ---------------------

def test_box5x5_vs_scipy():
    rng = np.random.default_rng(2)
    img = rng.integers(0, 1_040_401, size=(11, 9)).astype(np.float64)
    for border, c in (("replicate", 0.0), ("constant", 0.0), ("constant", 3.5)):
        mode, cval = _nd_mode(border, c)
        assert np.array_equal(oracle.box5x5_f64(img, border, c),
                              nd.correlate(img, np.ones((5, 5)), mode=mode, cval=cval))


def _harris(img, k=0.04, border="replicate"):
    gx, gy = oracle.sobel3x3(img, border)
    sxx = oracle.box5x5_f64(oracle.multiply_f64(gx, gx), border)
    syy = oracle.box5x5_f64(oracle.multiply_f64(gy, gy), border)
    sxy = oracle.box5x5_f64(oracle.multiply_f64(gx, gy), border)
    return oracle.harris_response(sxx, syy, sxy, k), (sxx, syy, sxy)


def test_harris_response_closed_forms():
    # constant image: no gradient, R = 0 everywhere, threshold gives 0
    r, _ = _harris(np.full((12, 12), 90, np.uint8))
    assert not r.any()
    # straight vertical edge: gy = 0 so det = 0 and R = -k * Sxx^2 <= 0
    img = np.zeros((16, 16), np.uint8)
    img[:, 8:] = 200
    r, (sxx, syy, sxy) = _harris(img)
    assert not syy.any() and not sxy.any()
    assert np.allclose(r, -0.04 * sxx ** 2) and r.max() <= 0
    # checkerboard corner: both gradients large, R far above 1e6
    img = np.full((32, 32), 40, np.uint8)
    img[8:16, 16:24] = 215
    img[16:24, 8:16] = 215
    r, _ = _harris(img)
    assert r[16, 16] > 1e10
    assert oracle.threshold(r, 1e6)[16, 16] == 255
    # the response formula itself on a hand-made tensor
    s = np.array([[4.0]]), np.array([[9.0]]), np.array([[2.0]])
    assert oracle.harris_response(*s, k=0.04)[0, 0] == pytest.approx(4 * 9 - 4 - 0.04 * 169)


def test_multiply_exact():
    a = np.array([[-1020, 1020, 7]], np.int16)
    assert oracle.multiply_f64(a, a).tolist() == [[1040400.0, 1040400.0, 49.0]]


# ---- graph executor ---------------------------------------------------------

def test_graph_executor_matches_composition():
    f = synth.uyvy_image(20, 10, seed=3)
    g = oracle.Graph()
    g.add("channel_extract_y", ["uyvy"], ["y"])
    g.add("gaussian3x3", ["y"], ["g"])
    g.add("sobel3x3", ["g"], ["gx", "gy"])
    g.add("magnitude", ["gy", "gy"], ["m"])
    g.add("threshold", ["m"], ["out"], thresh=100)
    env = oracle.run(g, {"uyvy": f})
    y = f[:, 1::2]
    gx, gy = oracle.sobel3x3(oracle.gaussian3x3(y))
    assert np.array_equal(env["out"], oracle.threshold(oracle.magnitude(gy, gy), 100))


def test_valid_masks_undefined_grows_by_radius():
    g = oracle.Graph()
    g.add("gaussian3x3", ["in"], ["g"], border="undefined")
    g.add("sobel3x3", ["g"], ["gx", "gy"], border="undefined")
    g.add("magnitude", ["gx", "gy"], ["m"])
    m = oracle.valid_masks(g, {"in": (10, 12)})["m"]
    assert m.sum() == (10 - 4) * (12 - 4) and m[2:-2, 2:-2].all()
    g2 = oracle.Graph()
    g2.add("gaussian3x3", ["in"], ["g"], border="replicate")
    g2.add("sobel3x3", ["g"], ["gx", "gy"], border="undefined")
    assert oracle.valid_masks(g2, {"in": (10, 12)})["gx"].sum() == 8 * 10


def test_cycle_rejected():
    g = oracle.Graph()
    g.add("gaussian3x3", ["a"], ["b"])
    g.add("gaussian3x3", ["b"], ["a"])
    with pytest.raises(ValueError):
        oracle.run(g, {})


@pytest.mark.parametrize("h,w", [(1, 1), (1, 3), (2, 3), (4, 2), (3, 7)])
def test_repeat_border_on_images_smaller_than_the_window(h, w):
    """REPEAT tiles the image periodically, also when the window wraps
    around more than once: the 5x5 Gaussian and Box3x3 equal plain windowed
    sums over numpy's periodic padding, and the wrapped window of NonMax
    sees copies of the pixel itself on one-pixel axes."""
    rng = np.random.default_rng(h * 10 + w)
    img = rng.integers(0, 256, size=(h, w), dtype=np.uint8)
    pad = np.pad(img.astype(np.int64), 2, mode="wrap")
    b = np.array([1, 4, 6, 4, 1])
    g = sum(b[j] * b[i] * pad[j:j + h, i:i + w] for j in range(5) for i in range(5)) >> 8
    assert np.array_equal(oracle.gaussian5x5(img, "repeat"), g)
    box = sum(pad[1 + j:1 + j + h, 1 + i:1 + i + w] for j in range(3) for i in range(3)) // 9
    assert np.array_equal(oracle.box3x3(img, "repeat"), box)
    if w == 1:  # the position left of the pixel is the pixel itself
        assert np.all(oracle.nonmax(img, 3, "repeat") == 0)

