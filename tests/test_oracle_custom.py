"""Pins of the oracle for user-defined point nodes (Section 5.1) against
numpy's own int32 arithmetic, closed forms and a library eigenvalue routine."""
import numpy as np
import pytest

from oracle import custom

RNG = np.random.default_rng(5)
A8 = RNG.integers(0, 256, (9, 13), dtype=np.uint8)
B8 = RNG.integers(0, 256, (9, 13), dtype=np.uint8)
S1 = RNG.integers(-32768, 32768, (9, 13), dtype=np.int16)
S2 = RNG.integers(-32768, 32768, (9, 13), dtype=np.int16)
S3 = RNG.integers(-32768, 32768, (9, 13), dtype=np.int16)


def test_products_wrap_like_numpy_int32():
    # numpy's int32 arrays wrap modulo 2^32 on overflow: an independent machine
    want = (S1.astype(np.int32) * S2.astype(np.int32) * S3.astype(np.int32)) - S1.astype(np.int32)
    got_s16 = custom.evaluate("a * b * c - a", [S1, S2, S3], np.int16)
    assert np.array_equal(got_s16, np.clip(want, -32768, 32767).astype(np.int16))
    # (-2^15)^2 * 2 = 2^31 wraps to -2^31, which saturates low rather than high
    one = lambda v: np.array([[v]], np.int16)
    assert custom.evaluate("a * b * c", [one(-32768), one(-32768), one(2)], np.int16).tolist() == [[-32768]]
    assert custom.evaluate("-(a * b * c)", [one(-32768), one(-32768), one(2)], np.int16).tolist() == [[-32768]]


def test_division_truncates_toward_zero_and_by_zero_gives_zero():
    x = np.array([[7, -7, 7, -7, 0, 5, -32768]], np.int16)
    y = np.array([[2, 2, -2, -2, 3, 0, -1]], np.int16)
    got = custom.evaluate("a / b", [x, y], np.int16)
    assert got.tolist() == [[3, -3, -3, 3, 0, 0, 32767]]  # 32768 saturates
    big = custom.evaluate("(a * 65536) / b", [np.array([[-32768]], np.int16), np.array([[-1]], np.int16)],
                          np.int16)
    assert big.tolist() == [[-32768]]  # -2^31 / -1 wraps to -2^31
    # against C-style division computed by numpy's trunc of the exact float quotient
    q = np.trunc(S1.astype(np.float64) / np.where(S2 == 0, 1, S2)).astype(np.int64)
    assert np.array_equal(custom.evaluate("a / b", [S1, S2], np.int16), np.clip(q, -32768, 32767))


def test_precedence_and_functions():
    a, b = A8.astype(np.int64), B8.astype(np.int64)
    assert np.array_equal(custom.evaluate("a - b * 2 + -a", [A8, B8], np.int16), a - 2 * b - a)
    assert np.array_equal(custom.evaluate("(a - b) * 2", [A8, B8], np.int16), np.clip((a - b) * 2, -32768, 32767))
    assert np.array_equal(custom.evaluate("max(a, b)", [A8, B8], np.uint8), np.maximum(A8, B8))
    assert np.array_equal(custom.evaluate("abs(a - b)", [A8, B8], np.uint8),
                          np.maximum(A8, B8) - np.minimum(A8, B8))
    assert np.array_equal(custom.evaluate("clamp(a, 40, 200)", [A8], np.uint8), np.clip(A8, 40, 200))
    assert np.array_equal(custom.evaluate("sel(gt(a, b), a, 0)", [A8, B8], np.uint8), np.where(A8 > B8, A8, 0))
    assert np.array_equal(custom.evaluate("a + b", [A8, B8], np.uint8),
                          np.clip(a + b, 0, 255).astype(np.uint8))


def test_float_kernel_min_eigenvalue_matches_eigvalsh():
    """The Shi-Tomasi response: the smaller eigenvalue of [[sxx, sxy], [sxy, syy]]."""
    rng = np.random.default_rng(1)
    sxx, syy = rng.uniform(0, 1e6, (2, 40, 30))
    sxy = rng.uniform(-1e6, 1e6, (40, 30))
    got = custom.evaluate("(a + b) / 2 - sqrt((a - b) * (a - b) / 4 + c * c)", [sxx, syy, sxy], np.float64)
    m = np.stack([np.stack([sxx, sxy], -1), np.stack([sxy, syy], -1)], -2)
    want = np.linalg.eigvalsh(m)[..., 0]
    assert np.allclose(got, want, rtol=0, atol=1e-9 * np.abs(m).max())


@pytest.mark.parametrize("expr,nin,flt", [("a ** 2", 1, False), ("a % 3", 1, False), ("a // 2", 1, False),
                                          ("sqrt(a)", 1, False), ("a + 1.5", 1, False), ("d", 1, False),
                                          ("b", 1, False), ("min(a)", 1, False), ("foo(a)", 1, False),
                                          ("a > 1", 1, False), ("a +", 1, False), ("4294967296", 1, False),
                                          ("a if b else c", 3, False), ("[a]", 1, True)])
def test_grammar_rejects(expr, nin, flt):
    with pytest.raises(ValueError):
        custom.check(expr, nin, flt)


def test_float_kernel_needs_f32_output():
    with pytest.raises(ValueError):
        custom.evaluate("a", [np.zeros((2, 2))], np.uint8)


SOBEL_X = "a[1, -1] + 2 * a[1, 0] + a[1, 1] - a[-1, -1] - 2 * a[-1, 0] - a[-1, 1]"
GAUSS3 = "(a[-1, -1] + 2 * a[0, -1] + a[1, -1] + 2 * a[-1, 0] + 4 * a + 2 * a[1, 0] + a[-1, 1] + 2 * a[0, 1] + a[1, 1]) / 16"


@pytest.mark.parametrize("border,c", [("replicate", 0), ("constant", 0), ("constant", 77), ("mirror", 0),
                                      ("repeat", 0)])
@pytest.mark.parametrize("h,w", [(9, 13), (2, 3), (1, 5)])
def test_local_kernel_matches_the_c_oracle_stencils(border, c, h, w):
    """A user local kernel written as the Sobel gx or the Gaussian3x3 stencil
    equals the C oracle's node at every border (numpy padding here, the C
    oracle's own border fetch there)."""
    import oracle
    img = np.random.default_rng(h * w).integers(0, 256, (h, w), dtype=np.uint8)
    gx, _ = oracle.sobel3x3(img, border, c)
    assert np.array_equal(custom.evaluate_local(SOBEL_X, img, np.int16, border, c), gx)
    assert np.array_equal(custom.evaluate_local(GAUSS3, img, np.uint8, border, c), oracle.gaussian3x3(img, border, c))


def test_local_kernel_grammar():
    with pytest.raises(ValueError):
        custom.check("a[3, 0]", 1, False, local=True)
    with pytest.raises(ValueError):
        custom.check("a[1]", 1, False, local=True)
    with pytest.raises(ValueError):
        custom.check("a[1, 0]", 1, False, local=False)
    with pytest.raises(ValueError):
        custom.check("b[1, 0]", 2, False, local=True)
    custom.check("a[-2, 2] - a", 1, False, local=True)
