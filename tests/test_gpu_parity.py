"""GPU parity: the HIP path against the CPU oracle, element by element, on
seeded inputs.  Integer outputs must be bit-exact, Phase within one level
(circular), the corner response's threshold exact outside the 1e-5 relative
tolerance band.  Sizes span several work items and ragged tails."""
import numpy as np
import pytest

import oracle
import paper_2008_11476_amd as hvx
import synth
from tests import graphspec as gs
from tests.gpu_util import compare, log, run_spec

pytestmark = pytest.mark.gpu

# MIRROR and REPEAT last: the slices BORDERS[:2] / [:3] keep the modes the hand-fused kernels implement
BORDERS = [("replicate", 0), ("constant", 0), ("constant", 77), ("undefined", 0), ("mirror", 0), ("repeat", 0)]


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = hvx.hvx_context_create(0)
    yield c
    hvx.hvx_context_release(c)


# ---- single operators, node by node (generic tile kernel) ------------------

LOCAL_U8 = ["gaussian3x3", "gaussian5x5", "box3x3", "dilate3x3", "erode3x3", "median3x3"]
SIZES = [(1, 1), (2, 3), (7, 5), (17, 13), (67, 45), (300, 70)]


@pytest.mark.parametrize("op", LOCAL_U8)
@pytest.mark.parametrize("w,h", SIZES)
@pytest.mark.parametrize("border", BORDERS)
def test_local_u8(ctx, op, w, h, border):
    log("local %s %dx%d %s" % (op, w, h, border))
    img = synth.edge_image(w, h, seed=w + 7 * h)
    spec = gs.Spec([gs.N(op, ["in"], ["out"], *border)], {"in": img}, {"out": np.uint8})
    got, _ = run_spec(spec, ctx, fusion=False, specialize=False)
    compare(spec, got, spec.run_oracle())


NL_MASKS = {"box3": np.ones((3, 3)), "cross3": np.array([[0, 1, 0], [1, 1, 1], [0, 1, 0]]),
            "disk5": np.array([[0, 1, 1, 1, 0]] + [[1] * 5] * 3 + [[0, 1, 1, 1, 0]]),
            "custom5x3": np.array([[1, 0, 0, 1, 1], [0, 1, 1, 0, 1], [1, 1, 0, 0, 0]]),
            "pair1x3": np.array([[1, 0, 1]])}


@pytest.mark.parametrize("mask", sorted(NL_MASKS))
@pytest.mark.parametrize("func", ["median", "min", "max"])
@pytest.mark.parametrize("border", BORDERS)
def test_nonlinear_filter(ctx, mask, func, border):
    """NonLinearFilter, node by node (one-operator kernel) and fused behind a
    Gaussian3x3 with a Threshold after it (generic tile kernel)."""
    w, h = 67, 45
    img = synth.edge_image(w, h, seed=len(mask) + len(func))
    m = NL_MASKS[mask]
    log("nonlinear %s %s %s" % (mask, func, border))
    one = gs.Spec([gs.N("nonlinear", ["in"], ["out"], *border, params={"mask": m, "func": func})],
                  {"in": img}, {"out": np.uint8})
    got, _ = run_spec(one, ctx, fusion=False)
    compare(one, got, one.run_oracle())
    chain = gs.Spec([gs.N("gaussian3x3", ["in"], ["g"], *border),
                     gs.N("nonlinear", ["g"], ["f"], *border, params={"mask": m, "func": func}),
                     gs.N("threshold", ["f"], ["out"], params={"thresh": 110})],
                    {"in": img}, {"f": np.uint8, "out": np.uint8})
    got, g = run_spec(chain, ctx)
    assert hvx.hvx_graph_query(g, hvx.HVX_QUERY_NUM_KERNELS) == (1 if border[0] != "repeat" else 3)
    compare(chain, got, chain.run_oracle())


def test_nonlinear_filter_rejects_bad_masks(ctx):
    g = hvx.hvx_graph_create(ctx)
    ab, av = hvx.alloc_image(8, 8, hvx.HVX_DF_U8)
    ob, ov = hvx.alloc_image(8, 8, hvx.HVX_DF_U8)
    a = hvx.image_from_tensor(ctx, av, hvx.HVX_DF_U8)
    o = hvx.image_from_tensor(ctx, ov, hvx.HVX_DF_U8)
    for bad in (np.ones((2, 3)), np.ones((7, 7)), np.zeros((3, 3))):
        with pytest.raises(hvx.HvxError):
            hvx.hvx_nonlinear_filter_node(g, hvx.HVX_NONLINEAR_MEDIAN, a, bad, o, ctx=ctx)
    with pytest.raises(hvx.HvxError):
        hvx.hvx_nonlinear_filter_node(g, 3, a, np.ones((3, 3)), o, ctx=ctx)
    hvx.hvx_release_graph(g)


@pytest.mark.parametrize("win", [3, 5])
@pytest.mark.parametrize("border", BORDERS)
@pytest.mark.parametrize("w,h", [(67, 45), (5, 3), (1100, 19)])
def test_nonmax_u8(ctx, win, border, w, h):
    """NonMaxSuppression on U8, node by node (one-operator kernel) on a
    smoothed edge image (plateaus) and on four-level noise (ties everywhere),
    and fused behind a Gaussian3x3 with its output also thresholded (generic
    tile kernel)."""
    log("nonmax u8 win %d %s %dx%d" % (win, border, w, h))
    for img in (synth.edge_image(w, h, seed=win + w), synth.uniform_u8(w, h, seed=win + h) // 64):
        one = gs.Spec([gs.N("nonmax", ["in"], ["out"], *border, params={"win": win})], {"in": img},
                      {"out": np.uint8})
        got, _ = run_spec(one, ctx, fusion=False)
        compare(one, got, one.run_oracle())
    img = synth.edge_image(w, h, seed=win)
    chain = gs.Spec([gs.N("gaussian3x3", ["in"], ["g"], *border),
                     gs.N("nonmax", ["g"], ["n"], *border, params={"win": win}),
                     gs.N("threshold", ["n"], ["out"], params={"thresh": 90})],
                    {"in": img}, {"n": np.uint8, "out": np.uint8})
    got, g = run_spec(chain, ctx)
    assert hvx.hvx_graph_query(g, hvx.HVX_QUERY_NUM_KERNELS) == (1 if border[0] != "repeat" else 3)
    compare(chain, got, chain.run_oracle())


@pytest.mark.parametrize("win", [3, 5])
@pytest.mark.parametrize("border", [("replicate", 0), ("constant", -7), ("constant", 0), ("undefined", 0),
                                    ("mirror", 0), ("repeat", 0)])
def test_nonmax_s16(ctx, win, border):
    """NonMaxSuppression on S16: on the Sobel gx of an edge image, fused with
    the Sobel into one kernel and node by node, and on narrow-range S16 noise
    (many ties, negative values)."""
    w, h = 131, 37
    log("nonmax s16 win %d %s" % (win, border))
    img = synth.edge_image(w, h, seed=win)
    spec = gs.Spec([gs.N("sobel3x3", ["in"], ["gx", None]),
                    gs.N("nonmax", ["gx"], ["out"], *border, params={"win": win})],
                   {"in": img}, {"out": np.int16})
    env = spec.run_oracle()
    got, g = run_spec(spec, ctx)
    assert hvx.hvx_graph_query(g, hvx.HVX_QUERY_NUM_KERNELS) == (1 if border[0] != "repeat" else 2)
    compare(spec, got, env)
    unf, _ = run_spec(spec, ctx, fusion=False)
    compare(spec, unf, env)
    noise = synth.uniform_s16(w, h, seed=win, lo=-12, hi=3)
    one = gs.Spec([gs.N("nonmax", ["in"], ["out"], *border, params={"win": win})], {"in": noise},
                  {"out": np.int16})
    got, _ = run_spec(one, ctx, fusion=False)
    compare(one, got, one.run_oracle())


@pytest.mark.parametrize("w,h", [(1, 1), (3, 2), (67, 45), (130, 21)])
def test_repeat_border_fused_and_split(ctx, w, h):
    """REPEAT on operators that read the graph input stays fused (the tile
    loads its halo from the periodic positions); REPEAT on an operator that
    reads an intermediate splits the group into single operators.  Both
    against the oracle, on images down to one pixel (windows wrapping more
    than once)."""
    img = synth.edge_image(w, h, seed=w * h)
    rp = ("repeat", 0)
    fused = gs.Spec([gs.N("gaussian5x5", ["in"], ["g"], *rp), gs.N("box3x3", ["in"], ["b"], *rp),
                     gs.N("add", ["g", "b"], ["s"]), gs.N("threshold", ["s"], ["out"], params={"thresh": 200})],
                    {"in": img}, {"s": np.uint8, "out": np.uint8})
    log("repeat fused %dx%d" % (w, h))
    got, g = run_spec(fused, ctx)
    assert hvx.hvx_graph_query(g, hvx.HVX_QUERY_NUM_KERNELS) == 1
    compare(fused, got, fused.run_oracle())
    split = gs.Spec([gs.N("gaussian3x3", ["in"], ["g"]), gs.N("dilate3x3", ["g"], ["d"], *rp),
                     gs.N("sobel3x3", ["d"], ["gx", "gy"], *rp), gs.N("magnitude", ["gx", "gy"], ["out"])],
                    {"in": img}, {"out": np.int16})
    log("repeat split %dx%d" % (w, h))
    got, g = run_spec(split, ctx)
    assert hvx.hvx_graph_query(g, hvx.HVX_QUERY_NUM_KERNELS) == 5  # Sobel lowers to two local operators
    compare(split, got, split.run_oracle())


def test_nonmax_rejects_bad_windows(ctx):
    g = hvx.hvx_graph_create(ctx)
    ab, av = hvx.alloc_image(8, 8, hvx.HVX_DF_U8)
    ob, ov = hvx.alloc_image(8, 8, hvx.HVX_DF_U8)
    a = hvx.image_from_tensor(ctx, av, hvx.HVX_DF_U8)
    o = hvx.image_from_tensor(ctx, ov, hvx.HVX_DF_U8)
    for bad in (0, 1, 4, 7):
        with pytest.raises(hvx.HvxError):
            hvx.hvx_non_max_suppression_node(g, a, bad, o, ctx=ctx)
    hvx.hvx_release_graph(g)


@pytest.mark.parametrize("border", [("replicate", 0), ("constant", 30), ("undefined", 0), ("mirror", 0),
                                    ("repeat", 0)])
@pytest.mark.parametrize("w,h", [(301, 77), (64, 9)])
def test_morphology_chain_fused(ctx, border, w, h):
    """Gaussian3x3 -> Median3x3 -> Dilate3x3 -> Erode3x3 -> Threshold as one
    fused kernel (intermediates in LDS, borders node by node), the median also
    as an output; against the oracle and the unfused path."""
    img = synth.edge_image(w, h, seed=w + h)
    spec = gs.Spec([gs.N("gaussian3x3", ["in"], ["g"], *border), gs.N("median3x3", ["g"], ["m"], *border),
                    gs.N("dilate3x3", ["m"], ["d"], *border), gs.N("erode3x3", ["d"], ["e"], *border),
                    gs.N("threshold", ["e"], ["out"], params={"thresh": 100})],
                   {"in": img}, {"m": np.uint8, "out": np.uint8})
    env = spec.run_oracle()
    log("morphology chain %dx%d %s" % (w, h, border))
    got, g = run_spec(spec, ctx)
    assert hvx.hvx_graph_query(g, hvx.HVX_QUERY_NUM_KERNELS) == (1 if border[0] != "repeat" else 5)
    compare(spec, got, env)
    unf, _ = run_spec(spec, ctx, fusion=False)
    compare(spec, unf, env)


@pytest.mark.parametrize("w,h", SIZES)
@pytest.mark.parametrize("border", BORDERS)
def test_sobel_s16(ctx, w, h, border):
    log("sobel %dx%d %s" % (w, h, border))
    img = synth.edge_image(w, h, seed=3 * w + h)
    spec = gs.Spec([gs.N("sobel3x3", ["in"], ["gx", "gy"], *border)], {"in": img},
                   {"gx": np.int16, "gy": np.int16})
    got, _ = run_spec(spec, ctx, fusion=False)
    compare(spec, got, spec.run_oracle())


def test_magnitude_and_phase_exhaustive_range(ctx):
    """Every (gx, gy) in the Sobel range [-1020, 1020]^2 plus S16 extremes."""
    r = np.arange(-1020, 1021, dtype=np.int16)
    gx, gy = np.meshgrid(r, r)
    ext = synth.uniform_s16(2041, 8, seed=9)
    gx = np.concatenate([gx, ext, np.full((1, 2041), -32768, np.int16)])
    gy = np.concatenate([gy, synth.uniform_s16(2041, 8, seed=10), np.full((1, 2041), -32768, np.int16)])
    log("magnitude/phase exhaustive %s" % (gx.shape,))
    spec = gs.Spec([gs.N("magnitude", ["gx", "gy"], ["m"]), gs.N("phase", ["gx", "gy"], ["p"])],
                   {"gx": gx, "gy": gy}, {"m": np.int16, "p": np.uint8})
    got, _ = run_spec(spec, ctx, fusion=False)
    compare(spec, got, spec.run_oracle(), phase_names=("p",))


@pytest.mark.parametrize("dtype,thresh", [(np.uint8, 100), (np.uint8, 99.5), (np.int16, -3), (np.int16, 1000.0),
                                          (np.float32, 12.25)])
def test_threshold(ctx, dtype, thresh):
    log("threshold %s %s" % (np.dtype(dtype), thresh))
    rng = np.random.default_rng(4)
    if dtype == np.float32:
        img = rng.normal(12, 3, size=(37, 129)).astype(np.float32)
        img[0, :5] = [12.25, np.nextafter(np.float32(12.25), np.float32(20)), -1e30, 1e30, 0]
    elif dtype == np.int16:
        img = synth.uniform_s16(129, 37, seed=5, lo=-2000, hi=2000)
    else:
        img = synth.uniform_u8(129, 37, seed=6)
    spec = gs.Spec([gs.N("threshold", ["in"], ["out"], params={"thresh": thresh, "true_v": 9, "false_v": 200})],
                   {"in": img}, {"out": np.uint8})
    env = spec.run_oracle() if dtype != np.float32 else None
    if env is None:  # the oracle reads real-valued images as double
        env = oracle.run(spec.oracle_graph(), {"in": img.astype(np.float64)})
    got, _ = run_spec(spec, ctx, fusion=False)
    compare(spec, got, env)


@pytest.mark.parametrize("ta,tb,to,policy", [("u8", "u8", "u8", "saturate"), ("u8", "u8", "u8", "wrap"),
                                             ("u8", "s16", "s16", "saturate"), ("s16", "s16", "s16", "wrap"),
                                             ("s16", "s16", "s16", "saturate")])
def test_add(ctx, ta, tb, to, policy):
    log("add %s %s %s %s" % (ta, tb, to, policy))
    mk = {"u8": lambda s: synth.uniform_u8(77, 19, seed=s), "s16": lambda s: synth.uniform_s16(77, 19, seed=s)}
    spec = gs.Spec([gs.N("add", ["a", "b"], ["out"], params={"policy": policy, "out_dtype": to})],
                   {"a": mk[ta](1), "b": mk[tb](2)}, {"out": np.uint8 if to == "u8" else np.int16})
    got, _ = run_spec(spec, ctx, fusion=False)
    compare(spec, got, spec.run_oracle())


@pytest.mark.parametrize("mask,scale,out", [
    (np.array([[0, 1, 0], [1, -4, 1], [0, 1, 0]]), 1, np.int16),   # Laplacian test mask
    (np.array([[1, -2, 3], [0, 4, -5], [6, 0, -1]]), 2, np.int16),
    (np.array([[1, 2, 1], [2, 4, 2], [1, 2, 1]]), 16, np.uint8),
    (np.arange(15).reshape(3, 5) - 7, 4, np.int16),
    (np.arange(25).reshape(5, 5) - 12, 1, np.uint8)])
@pytest.mark.parametrize("border", BORDERS[:3])
def test_convolve(ctx, mask, scale, out, border):
    log("convolve %s scale %d %s" % (mask.shape, scale, border))
    img = synth.edge_image(83, 41, seed=8)
    spec = gs.Spec([gs.N("convolve", ["in"], ["out"], *border,
                         params={"coeffs": mask, "scale": scale, "out_dtype": "u8" if out == np.uint8 else "s16"})],
                   {"in": img}, {"out": out})
    got, _ = run_spec(spec, ctx, fusion=False)
    compare(spec, got, spec.run_oracle())


def test_channel_extract(ctx):
    f = synth.uyvy_image(98, 33, seed=2)
    log("channel extract")
    spec = gs.Spec([gs.N("channel_extract_y", ["in"], ["out"])], {"in": f}, {"out": np.uint8}, uyvy=("in",))
    got, _ = run_spec(spec, ctx, fusion=False)
    compare(spec, got, spec.run_oracle())


# ---- fused graphs ---------------------------------------------------------------

EDGE_SIZES = [(1, 1), (5, 3), (15, 2), (16, 16), (17, 9), (100, 37), (992, 20), (993, 21), (1000, 64),
              (1985, 33), (2000, 70), (640, 480)]


@pytest.mark.parametrize("w,h", EDGE_SIZES)
@pytest.mark.parametrize("phase", [False, True])
def test_edge_fused_fast(ctx, w, h, phase):
    img = synth.edge_image(w, h, seed=w * 3 + h)
    spec = gs.edge_spec(img, phase=phase)
    env = spec.run_oracle()
    for rows in (0, 4, 7):
        log("edge fast %dx%d phase=%s rows=%d" % (w, h, phase, rows))
        got, g = run_spec(spec, ctx, rows=rows)
        assert hvx.hvx_graph_query(g, hvx.HVX_QUERY_KERNEL_KIND) == 1
        compare(spec, got, env, phase_names=("ph",))


@pytest.mark.parametrize("b0", BORDERS)
@pytest.mark.parametrize("b1", BORDERS)
def test_edge_fused_borders(ctx, b0, b1):
    w, h = 1001, 45
    img = synth.edge_image(w, h, seed=11)
    spec = gs.edge_spec(img, phase=True, b0=b0, b1=b1)
    env = spec.run_oracle()
    for specialize in (True, False):
        log("edge borders %s %s specialize=%s" % (b0, b1, specialize))
        got, _ = run_spec(spec, ctx, specialize=specialize, rows=8)
        compare(spec, got, env, phase_names=("ph",))


@pytest.mark.parametrize("thresh", [-1, 0, 1, 99.5, 100, 180, 180.5, 181, 1442, 1443, 40000])
@pytest.mark.parametrize("phase", [False, True])
def test_edge_thresholds(ctx, thresh, phase):
    """Bounds u(u-1) up to 32767 (threshold below 181) take the fused
    kernel's saturating 16-bit magnitude test, larger ones the 32-bit test;
    both sides of that switch and the extremes."""
    img = synth.edge_image(300, 40, seed=12)
    spec = gs.edge_spec(img, thresh=thresh, phase=phase)
    log("edge threshold %s phase %s" % (thresh, phase))
    got, _ = run_spec(spec, ctx)
    compare(spec, got, spec.run_oracle(), phase_names=("ph",) if phase else ())


@pytest.mark.parametrize("w,h", [(64, 48), (1003, 67)])
def test_edge_unfused_and_generic_match(ctx, w, h):
    img = synth.edge_image(w, h, seed=5)
    spec = gs.edge_spec(img, phase=True)
    env = spec.run_oracle()
    log("edge unfused %dx%d" % (w, h))
    unf, _ = run_spec(spec, ctx, fusion=False)
    gen, _ = run_spec(spec, ctx, specialize=False)
    fast, _ = run_spec(spec, ctx)
    compare(spec, unf, env, phase_names=("ph",))
    compare(spec, gen, env, phase_names=("ph",))
    assert np.array_equal(unf["out"], fast["out"]) and np.array_equal(gen["out"], fast["out"])
    # one phase function serves every kernel: Phase is bitwise equal too
    assert np.array_equal(unf["ph"], fast["ph"]) and np.array_equal(gen["ph"], fast["ph"])


@pytest.mark.parametrize("w,h", [(1, 1), (2, 3), (17, 9), (100, 37), (993, 21), (2000, 70)])
@pytest.mark.parametrize("border", BORDERS[:3])
def test_gauss5_fused(ctx, w, h, border):
    img = synth.edge_image(w, h, seed=w + h)
    spec = gs.gauss5_spec(img, border)
    log("gauss5 %dx%d %s" % (w, h, border))
    got, g = run_spec(spec, ctx, rows=5)
    assert hvx.hvx_graph_query(g, hvx.HVX_QUERY_KERNEL_KIND) == 3
    compare(spec, got, spec.run_oracle())


@pytest.mark.parametrize("w,h", [(2, 1), (18, 9), (100, 37), (994, 21), (1280, 72)])
@pytest.mark.parametrize("border", BORDERS[:2])
def test_uyvy_gauss5_fused(ctx, w, h, border):
    f = synth.uyvy_image(w, h, seed=w)
    spec = gs.uyvy_gauss5_spec(f, border)
    log("uyvy gauss5 %dx%d %s" % (w, h, border))
    got, g = run_spec(spec, ctx, rows=6)
    assert hvx.hvx_graph_query(g, hvx.HVX_QUERY_KERNEL_KIND) == 3
    compare(spec, got, spec.run_oracle())
    got2, _ = run_spec(spec, ctx, fusion=False)
    compare(spec, got2, spec.run_oracle())


@pytest.mark.parametrize("w,h", [(2, 2), (3, 5), (130, 41)])
@pytest.mark.parametrize("fusion", [True, False])
def test_corner_mirror(ctx, w, h, fusion):
    """The corner graph with MIRROR borders runs on the generic kernels (the
    F32 Box5x5 reads mirrored F32 products)."""
    img = synth.corner_image(w, h, seed=w + 1)
    spec = gs.corner_spec(img, b0=("mirror", 0), b1=("mirror", 0))
    env = spec.run_oracle()
    log("corner mirror %dx%d fusion=%s" % (w, h, fusion))
    got, g = run_spec(spec, ctx, fusion=fusion)
    assert hvx.hvx_graph_query(g, hvx.HVX_QUERY_KERNEL_KIND) == 0
    compare(spec, got, env, corner=True)


@pytest.mark.parametrize("w,h", [(13, 11), (200, 60), (1003, 45)])
@pytest.mark.parametrize("fusion", [True, False])
def test_corner(ctx, w, h, fusion):
    img = synth.corner_image(w, h, seed=w)
    spec = gs.corner_spec(img)
    env = spec.run_oracle()
    log("corner %dx%d fusion=%s" % (w, h, fusion))
    got, _ = run_spec(spec, ctx, fusion=fusion)
    compare(spec, got, env, corner=True)
    assert got["out"].max() == 255 or env["out"].max() == 0


def test_listing1_dce_on_off(ctx):
    f = synth.uyvy_image(130, 41, seed=4)
    spec = gs.listing1_spec(f)
    env = spec.run_oracle()
    log("listing 1 dce")
    a, _ = run_spec(spec, ctx, dce=True)
    b, _ = run_spec(spec, ctx, dce=False)
    c, _ = run_spec(spec, ctx, dce=True, fusion=False)
    compare(spec, a, env)
    assert np.array_equal(a["out"], b["out"]) and np.array_equal(a["out"], c["out"])


def test_fast_kernel_tile_shapes_bitwise_equal(ctx):
    """Every rows-per-item setting and both work mappings give the same bytes."""
    img = synth.edge_image(2100, 300, seed=21)
    spec = gs.edge_spec(img, phase=True)
    ref = None
    for rows in (1, 2, 3, 8, 16, 64, 300):
        for xcd in (True, False):
            log("tile shape rows=%d xcd=%s" % (rows, xcd))
            got, _ = run_spec(spec, ctx, rows=rows, xcd=xcd)
            if ref is None:
                ref = got
            assert np.array_equal(got["out"], ref["out"]) and np.array_equal(got["ph"], ref["ph"])


def test_autotune_keeps_results(ctx):
    img = synth.edge_image(1920, 1080, seed=0)
    spec = gs.edge_spec(img)
    log("autotune 1920x1080")
    got, g = run_spec(spec, ctx, autotune=True)
    compare(spec, got, spec.run_oracle())
