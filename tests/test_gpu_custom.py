"""GPU parity of user-defined point nodes (Section 5.1) and of the paper's
applications built with them (Unsharp, Tomasi; Section 6.1), against the
oracle.  Integer kernels bit-exact; float kernels within a relative
tolerance derived from the F32 arithmetic."""
import numpy as np
import pytest

import oracle
import paper_2008_11476_amd as hvx
import synth
from tests import graphspec as gs
from tests.gpu_util import compare, log, run_spec

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = hvx.hvx_context_create(0)
    yield c
    hvx.hvx_context_release(c)


# (expression, input dtypes, output dtype)
INT_KERNELS = [
    ("a + b", (np.uint8, np.uint8), np.uint8),
    ("a - b * 2 + -a", (np.uint8, np.uint8), np.int16),
    ("abs(a - b)", (np.int16, np.int16), np.int16),
    ("max(a, b) - min(a, b)", (np.uint8, np.int16), np.uint8),
    ("clamp(a * 3 / 2, 10, 200)", (np.uint8,), np.uint8),
    ("sel(gt(a, b), a, b / 3)", (np.int16, np.uint8), np.int16),
    ("a * b * c - a", (np.int16, np.int16, np.int16), np.int16),
    ("-(a * b * c)", (np.int16, np.int16, np.int16), np.int16),
    ("(a * 65536) / b", (np.int16, np.int16), np.int16),
    ("a / b + a / -7 - 2147483647", (np.int16, np.int16), np.int16),
    ("((((((a + 1) * 2 + 3) * 4 + 5) * 6 + 7) * 8 + b) / 5) - c", (np.uint8, np.uint8, np.uint8), np.int16),
]


def _inputs(dtypes, w, h, seed):
    out = {}
    for k, dt in enumerate(dtypes):
        if dt == np.uint8:
            out["abc"[k]] = synth.uniform_u8(w, h, seed=seed + k)
        else:
            # narrow values, zeros and the extremes so that division and wrap-around edges occur
            v = synth.uniform_s16(w, h, seed=seed + k, lo=-300, hi=300)
            v.flat[::7] = 0
            v.flat[3::11] = -32768
            v.flat[5::13] = 32767
            v.flat[2::17] = -1
            out["abc"[k]] = v
    return out


@pytest.mark.parametrize("expr,ins,out", INT_KERNELS)
@pytest.mark.parametrize("w,h", [(67, 45), (1, 1), (1029, 3)])
def test_integer_kernel(ctx, expr, ins, out, w, h):
    """Node by node (one-operator kernel) and fused with the nodes around it
    (generic tile kernel): bit-exact."""
    log("custom int %r %dx%d" % (expr, w, h))
    inputs = _inputs(ins, w, h, seed=len(expr) + w)
    names = list(inputs)
    one = gs.Spec([gs.N("custom_point", names, ["out"], params={"expr": expr, "out_dtype": out})], inputs,
                  {"out": out})
    got, _ = run_spec(one, ctx, fusion=False)
    compare(one, got, one.run_oracle())
    # fused: the first input smoothed first (a U8 first input only), the result thresholded
    if ins[0] == np.uint8:
        nodes = [gs.N("gaussian3x3", ["a"], ["g"]),
                 gs.N("custom_point", ["g"] + names[1:], ["r"], params={"expr": expr, "out_dtype": out}),
                 gs.N("threshold", ["r"], ["t"], params={"thresh": 20})]
        fused = gs.Spec(nodes, inputs, {"r": out, "t": np.uint8})
        got, g = run_spec(fused, ctx)
        assert hvx.hvx_graph_query(g, hvx.HVX_QUERY_NUM_KERNELS) == 1
        compare(fused, got, fused.run_oracle())


def _close(got, want, scale, rel=1e-5):
    bad = np.abs(got.astype(np.float64) - want) > rel * scale + 1e-6
    assert not bad.any(), "%d of %d differ beyond the tolerance, worst %g" % (
        bad.sum(), bad.size, np.abs(got - want)[bad].max())


def test_float_kernel_mixed_inputs(ctx):
    """F32 from S16 and F32 inputs: sqrt, division, min/max, sel."""
    w, h = 131, 29
    rng = np.random.default_rng(3)
    a = synth.uniform_s16(w, h, seed=1, lo=-2000, hi=2000)
    b = rng.uniform(-1e4, 1e4, (h, w)).astype(np.float32)
    c = rng.uniform(0.5, 100, (h, w)).astype(np.float32)
    expr = "sqrt(abs(b)) * 0.5 + a / c - max(min(a, b), -3.25) + sel(gt(a, 0), c, -c)"
    spec = gs.Spec([gs.N("custom_point", ["a", "b", "c"], ["out"], params={"expr": expr, "out_dtype": np.float32})],
                   {"a": a, "b": b, "c": c}, {"out": np.float32})
    log("custom float mixed")
    for fusion in (False, True):
        got, _ = run_spec(spec, ctx, fusion=fusion)
        want = spec.run_oracle()["out"]
        scale = np.sqrt(np.abs(b)) + np.abs(a / c) + np.abs(a) + np.abs(b) + c
        _close(got["out"], want, scale)


def unsharp_spec(img, k_num=3, k_den=2):
    """Unsharp masking (Section 6.1: one Gauss node and three point nodes):
    detail = in - blur, boost = detail * k, out = saturate(in + boost)."""
    return gs.Spec([gs.N("gaussian3x3", ["in"], ["blur"]),
                    gs.N("custom_point", ["in", "blur"], ["detail"], params={"expr": "a - b", "out_dtype": np.int16}),
                    gs.N("custom_point", ["detail"], ["boost"],
                         params={"expr": "a * %d / %d" % (k_num, k_den), "out_dtype": np.int16}),
                    gs.N("custom_point", ["in", "boost"], ["out"], params={"expr": "a + b", "out_dtype": np.uint8})],
                   {"in": img}, {"out": np.uint8})


@pytest.mark.parametrize("w,h", [(640, 480), (1920, 1080), (33, 7)])
def test_unsharp_application(ctx, w, h):
    img = synth.edge_image(w, h, seed=w)
    spec = unsharp_spec(img)
    env = spec.run_oracle()
    log("unsharp %dx%d" % (w, h))
    got, g = run_spec(spec, ctx)
    assert hvx.hvx_graph_query(g, hvx.HVX_QUERY_NUM_KERNELS) == 1
    compare(spec, got, env)
    unf, g2 = run_spec(spec, ctx, fusion=False)
    assert hvx.hvx_graph_query(g2, hvx.HVX_QUERY_NUM_KERNELS) == 4
    compare(spec, unf, env)


TOMASI = "(a + b) / 2 - sqrt((a - b) * (a - b) / 4 + c * c)"


def tomasi_spec(img, thresh=2e5):
    """Shi-Tomasi corners (Section 6.1): the corner graph with the smaller
    eigenvalue of the structure tensor as the response."""
    return gs.Spec([gs.N("sobel3x3", ["in"], ["gx", "gy"]),
                    gs.N("multiply_f32", ["gx", "gx"], ["pxx"]),
                    gs.N("multiply_f32", ["gy", "gy"], ["pyy"]),
                    gs.N("multiply_f32", ["gx", "gy"], ["pxy"]),
                    gs.N("box5x5_f32", ["pxx"], ["sxx"]),
                    gs.N("box5x5_f32", ["pyy"], ["syy"]),
                    gs.N("box5x5_f32", ["pxy"], ["sxy"]),
                    gs.N("custom_point", ["sxx", "syy", "sxy"], ["r"], params={"expr": TOMASI,
                                                                             "out_dtype": np.float32}),
                    gs.N("threshold", ["r"], ["out"], params={"thresh": thresh})],
                   {"in": img}, {"r": np.float32, "out": np.uint8})


@pytest.mark.parametrize("w,h", [(640, 480), (129, 37)])
def test_tomasi_application(ctx, w, h):
    """Response within 1e-5 of the terms' scale (the F32 box sums and the
    cancellation in the smaller eigenvalue), thresholded output exact outside
    that band."""
    img = synth.corner_image(w, h, seed=w)
    spec = tomasi_spec(img)
    env = spec.run_oracle()
    scale = np.abs(env["sxx"]) + np.abs(env["syy"]) + np.abs(env["sxy"])
    log("tomasi %dx%d" % (w, h))
    for fusion in (True, False):
        got, g = run_spec(spec, ctx, fusion=fusion)
        if fusion:
            assert hvx.hvx_graph_query(g, hvx.HVX_QUERY_NUM_KERNELS) == 1
        _close(got["r"], env["r"], scale)
        amb = np.abs(env["r"] - 2e5) <= 1e-5 * scale + 1e-3
        bad = (got["out"] != env["out"]) & ~amb
        assert not bad.any(), "%d thresholded pixels differ outside the band" % bad.sum()
        assert (env["out"] == 255).sum() > 0  # the workload has corners


def _graph_with_images(ctx, dfs):
    import torch
    g = hvx.hvx_graph_create(ctx)
    keep, ims = [], []
    for df in dfs:
        dt = {hvx.HVX_DF_U8: torch.uint8, hvx.HVX_DF_S16: torch.int16, hvx.HVX_DF_F32: torch.float32}[df]
        t = torch.zeros((8, 64), dtype=dt, device="cuda")
        keep.append(t)
        ims.append(hvx.hvx_image_from_ptr(ctx, 64, 8, df, t.data_ptr(), t.stride(0) * t.element_size()))
    return g, ims, keep


@pytest.mark.parametrize("expr,nin", [("a +", 1), ("a ** 2", 1), ("b", 1), ("foo(a)", 1), ("min(a)", 1),
                                      ("a % 2", 1), ("(a", 1), ("a b", 1), ("", 1),
                                      ("a+" * 20 + "a", 1), ("min(a, max(b, min(a, max(b, min(a, max(b, min(a, "
                                                               "max(b, min(a, b)))))))))", 2),
                                      ("1+2+3+4+5+6+7+8+9+a", 1)])
def test_custom_rejects_bad_expressions(ctx, expr, nin):
    g, ims, keep = _graph_with_images(ctx, [hvx.HVX_DF_U8] * (nin + 1))
    with pytest.raises(hvx.HvxError):
        hvx.hvx_custom_point_node(g, expr, ims[:nin], hvx.HVX_DF_U8, ims[nin], ctx=ctx)
    hvx.hvx_release_graph(g)


@pytest.mark.parametrize("expr,in_df,out_df", [("sqrt(a)", hvx.HVX_DF_U8, hvx.HVX_DF_U8),
                                               ("a * 0.5", hvx.HVX_DF_S16, hvx.HVX_DF_S16),
                                               ("a + 2147483648", hvx.HVX_DF_U8, hvx.HVX_DF_S16),
                                               ("a", hvx.HVX_DF_F32, hvx.HVX_DF_U8)])
def test_custom_format_errors_at_verify(ctx, expr, in_df, out_df):
    g, ims, keep = _graph_with_images(ctx, [in_df, out_df])
    hvx.hvx_custom_point_node(g, expr, ims[:1], out_df, ims[1], ctx=ctx)
    with pytest.raises(hvx.HvxError):
        hvx.hvx_graph_verify(g, ctx=ctx)
    hvx.hvx_release_graph(g)


FCHAIN = [(np.outer([1, 4, 6, 4, 1], [1, 4, 6, 4, 1]), 256),      # Gaussian 5x5
          (np.array([[0, -1, 0], [-1, 5, -1], [0, -1, 0]]), 1),    # sharpen 3x3
          (np.ones((5, 5), int), 32)]                              # box 5x5, scaled down


@pytest.mark.parametrize("w,h", [(640, 480), (131, 29)])
@pytest.mark.parametrize("border", [("replicate", 0), ("constant", 9), ("mirror", 0)])
def test_fchain_application(ctx, w, h, border):
    """FChain (Section 6.1): three convolution nodes in a row, U8 between
    them, fused into one kernel (footprint 2 + 1 + 2) and node by node."""
    img = synth.edge_image(w, h, seed=h)
    names = ["in", "c1", "c2", "out"]
    nodes = [gs.N("convolve", [names[k]], [names[k + 1]], *border,
                  params={"coeffs": m, "scale": s, "out_dtype": "u8"}) for k, (m, s) in enumerate(FCHAIN)]
    spec = gs.Spec(nodes, {"in": img}, {"c1": np.uint8, "c2": np.uint8, "out": np.uint8})
    env = spec.run_oracle()
    log("fchain %dx%d %s" % (w, h, border))
    got, g = run_spec(spec, ctx)
    assert hvx.hvx_graph_query(g, hvx.HVX_QUERY_NUM_KERNELS) == 1
    compare(spec, got, env)
    unf, _ = run_spec(spec, ctx, fusion=False)
    compare(spec, unf, env)


LOCAL_KERNELS = [
    ("a[1, -1] + 2 * a[1, 0] + a[1, 1] - a[-1, -1] - 2 * a[-1, 0] - a[-1, 1]", np.int16),   # Sobel gx
    ("(a[-1, -1] + 2 * a[0, -1] + a[1, -1] + 2 * a[-1, 0] + 4 * a + 2 * a[1, 0] + a[-1, 1] + 2 * a[0, 1]"
     " + a[1, 1]) / 16", np.uint8),                                                          # Gaussian3x3
    ("max(a[-2, -2], a[2, 2]) - min(a[0, -2], a[0, 2]) + a[-2, 1] / 3", np.int16),          # 5x5 reach
    ("sqrt(a[1, 0] * a[-1, 0] + 1) / 2 + a[0, -1] * 0.25", np.float32),                   # float kernel
]
GPU_BORDERS = [("replicate", 0), ("constant", 0), ("constant", 77), ("undefined", 0), ("mirror", 0), ("repeat", 0)]


@pytest.mark.parametrize("expr,out", LOCAL_KERNELS)
@pytest.mark.parametrize("border", GPU_BORDERS)
@pytest.mark.parametrize("w,h", [(67, 45), (3, 2)])
def test_local_kernel(ctx, expr, out, border, w, h):
    """User local kernels node by node (generic tile kernel) and fused behind
    a Gaussian3x3 with a threshold after them."""
    log("custom local %r %s %dx%d" % (expr[:30], border, w, h))
    img = synth.edge_image(w, h, seed=w + len(expr))
    one = gs.Spec([gs.N("custom_local", ["in"], ["out"], *border, params={"expr": expr, "out_dtype": out})],
                  {"in": img}, {"out": out})
    env = one.run_oracle()
    got, _ = run_spec(one, ctx, fusion=False)
    if out == np.float32:
        m = oracle.valid_masks(one.oracle_graph(), one.shapes())["out"]
        _close(got["out"][m], env["out"][m], 1 + np.abs(env["out"][m]))
    else:
        compare(one, got, env)
    nodes = [gs.N("gaussian3x3", ["in"], ["g"], *border),
             gs.N("custom_local", ["g"], ["r"], *border, params={"expr": expr, "out_dtype": out}),
             gs.N("threshold", ["r"], ["t"], params={"thresh": 20})]
    fused = gs.Spec(nodes, {"in": img}, {"r": out, "t": np.uint8})
    env = fused.run_oracle()
    got, g = run_spec(fused, ctx)
    if border[0] != "repeat":
        assert hvx.hvx_graph_query(g, hvx.HVX_QUERY_NUM_KERNELS) == 1
    if out == np.float32:
        m = oracle.valid_masks(fused.oracle_graph(), fused.shapes())["r"]
        _close(got["r"][m], env["r"][m], 1 + np.abs(env["r"][m]))
    else:
        compare(fused, got, env)


@pytest.mark.parametrize("expr", ["a[3, 0]", "a[1]", "a[1, 0", "b[1, 0]", "a[1.5, 0]", "a[12, 0]", "b"])
def test_local_kernel_rejects(ctx, expr):
    g, ims, keep = _graph_with_images(ctx, [hvx.HVX_DF_U8, hvx.HVX_DF_U8])
    with pytest.raises(hvx.HvxError):
        hvx.hvx_custom_local_node(g, expr, ims[0], hvx.HVX_DF_U8, ims[1], ctx=ctx)
    with pytest.raises(hvx.HvxError):  # offsets are not allowed in a point kernel
        hvx.hvx_custom_point_node(g, "a[1, 0]", ims[:1], hvx.HVX_DF_U8, ims[1], ctx=ctx)
    hvx.hvx_release_graph(g)
