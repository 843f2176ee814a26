"""GPU parity of the kernels generated per fused group (HVX_OPT_CODEGEN):
each graph runs with its generated kernels and with the tile interpreter;
both are compared with the oracle, and with each other bit for bit (the
generated kernels evaluate the same operator definitions, only with the
operators, formats and offsets fixed at compile time)."""
import numpy as np
import pytest

import oracle
import paper_2008_11476_amd as hvx
import synth
from tests import graphspec as gs
from tests.gpu_util import compare, log, run_spec
from tests.test_gpu_custom import FCHAIN, TOMASI, unsharp_spec
from tests.test_gpu_global_graph import _check_buffers

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = hvx.hvx_context_create(0)
    yield c
    hvx.hvx_context_release(c)


def _fchain(img, border):
    names = ["in", "c1", "c2", "out"]
    nodes = [gs.N("convolve", [names[k]], [names[k + 1]], *border,
                  params={"coeffs": m, "scale": s, "out_dtype": "u8"}) for k, (m, s) in enumerate(FCHAIN)]
    return gs.Spec(nodes, {"in": img}, {"c1": np.uint8, "c2": np.uint8, "out": np.uint8})


# Convolve masks that are outer products of a column and a row (the
# generated kernel sums window columns first): 5x3 with a zero weight, 5x5
# with a signed row, and 5x3 whose column sums exceed 24 bits
SEPARABLE = [(np.outer([1, -2, 0, 3, 1], [2, -1, 1]), 4, "u8"),
             (np.outer([1, 4, 6, 4, 1], [-1, -2, 0, 2, 1]), 16, "u8"),
             (np.outer([7000, -7000, 7000, -7000, 7000], [3, -1, 3]), 32768, "s16")]


# 3x3 and 3-row by 5-column rank-one masks (column sums over three rows)
SEPARABLE3 = [(np.outer([1, -2, 1], [3, 1, 3]), 2, "u8"),
              (np.outer([2, 5, 2], [1, 3, -6, 3, 1]), 8, "s16")]


def _separable(img, border, masks=SEPARABLE):
    names = ["in", "c1", "c2", "out"][:len(masks)] + ["out"]
    nodes = [gs.N("convolve", [names[k]], [names[k + 1]], *border, params={"coeffs": m, "scale": s, "out_dtype": d})
             for k, (m, s, d) in enumerate(masks)]
    outs = {n: np.uint8 for n in names[1:-1]}
    outs["out"] = np.int16
    return gs.Spec(nodes, {"in": img}, outs)


def _tomasi(img):
    return gs.Spec([gs.N("sobel3x3", ["in"], ["gx", "gy"]),
                    gs.N("multiply_f32", ["gx", "gx"], ["pxx"]),
                    gs.N("multiply_f32", ["gy", "gy"], ["pyy"]),
                    gs.N("multiply_f32", ["gx", "gy"], ["pxy"]),
                    gs.N("box5x5_f32", ["pxx"], ["sxx"]),
                    gs.N("box5x5_f32", ["pyy"], ["syy"]),
                    gs.N("box5x5_f32", ["pxy"], ["sxy"]),
                    gs.N("custom_point", ["sxx", "syy", "sxy"], ["r"], params={"expr": TOMASI,
                                                                             "out_dtype": np.float32}),
                    gs.N("threshold", ["r"], ["out"], params={"thresh": 2e5})],
                   {"in": img}, {"r": np.float32, "out": np.uint8})


def _morph(img, border):
    return gs.Spec([gs.N("gaussian3x3", ["in"], ["g"], *border),
                    gs.N("dilate3x3", ["g"], ["d"], *border),
                    gs.N("median3x3", ["d"], ["m"], *border),
                    gs.N("erode3x3", ["m"], ["out"], *border)],
                   {"in": img}, {"out": np.uint8})


def _nonlinear(img, border):
    mask = np.array([[0, 1, 0, 1, 0], [1, 1, 1, 1, 1], [0, 1, 1, 1, 0]], np.uint8)
    return gs.Spec([gs.N("box3x3", ["in"], ["b"], *border),
                    gs.N("nonlinear", ["b"], ["nl"], *border, params={"func": "median", "mask": mask}),
                    gs.N("nonmax", ["nl"], ["out"], *border, params={"win": 3})],
                   {"in": img}, {"out": np.uint8})


def _laplace_float(img, border):
    return gs.Spec([gs.N("gaussian5x5", ["in"], ["g"], *border),
                    gs.N("custom_local", ["g"], ["lap"], *border,
                         params={"expr": "a[1, 0] + a[-1, 0] + a[0, 1] + a[0, -1] - 4 * a", "out_dtype": np.int16}),
                    gs.N("custom_point", ["lap", "in"], ["f"],
                         params={"expr": "sqrt(abs(a) * 0.5 + b) / 3", "out_dtype": np.float32}),
                    gs.N("threshold", ["f"], ["out"], params={"thresh": 2.5})],
                   {"in": img}, {"lap": np.int16, "f": np.float32, "out": np.uint8})


def _point_chain(a, b):
    return gs.Spec([gs.N("add", ["a", "b"], ["s"], params={"policy": "wrap"}),
                    gs.N("custom_point", ["s", "a", "b"], ["t"], params={"expr": "a * 3 - b / (c + 1)",
                                                                       "out_dtype": np.int16}),
                    gs.N("threshold", ["t"], ["out"], params={"thresh": 40})],
                   {"a": a, "b": b}, {"t": np.int16, "out": np.uint8})


def _edge_phase(img, b0, b1):
    return gs.edge_spec(img, phase=True, b0=b0, b1=b1)


def _uyvy(frame, border):
    return gs.Spec([gs.N("channel_extract_y", ["in"], ["y"]), gs.N("gaussian5x5", ["y"], ["g"], *border),
                    gs.N("sobel3x3", ["g"], ["gx", "gy"], *border), gs.N("magnitude", ["gx", "gy"], ["out"])],
                   {"in": frame}, {"out": np.int16}, uyvy=("in",))


def _s16_local(img, border):
    return gs.Spec([gs.N("sobel3x3", ["in"], ["gx", "gy"], *border),
                    gs.N("nonmax", ["gx"], ["n"], *border, params={"win": 5}),
                    gs.N("add", ["n", "gy"], ["out"], params={"policy": "saturate", "out_dtype": "s16"})],
                   {"in": img}, {"out": np.int16})


def _mixed_borders(img, b0, b1):
    """One value read by local operators with different borders (the
    generated kernel's edge tiles then read through each operator's rule)."""
    return gs.Spec([gs.N("gaussian3x3", ["in"], ["g"], *b0),
                    gs.N("box3x3", ["in"], ["b"], *b1),
                    gs.N("dilate3x3", ["g"], ["d"], *b1),
                    gs.N("median3x3", ["g"], ["m"], *b0),
                    gs.N("add", ["d", "b"], ["s"], params={"policy": "wrap"}),
                    gs.N("add", ["s", "m"], ["out"], params={"policy": "saturate"})],
                   {"in": img}, {"out": np.uint8})


BORDERS = [("replicate", 0), ("constant", 0), ("constant", 77), ("undefined", 0), ("mirror", 0)]
SIZES = [(129, 37), (1, 1), (640, 480), (3, 2)]


def _cases():
    out = []
    for w, h in SIZES:
        img = synth.edge_image(w, h, seed=w + h)
        out.append(("unsharp", (w, h), lambda img=img: unsharp_spec(img)))
        out.append(("tomasi", (w, h), lambda w=w, h=h: _tomasi(synth.corner_image(w, h, seed=w))))
        out.append(("point_chain", (w, h), lambda w=w, h=h: _point_chain(synth.uniform_u8(w, h, seed=3),
                                                                        synth.uniform_u8(w, h, seed=4))))
        for b in BORDERS:
            out.append(("fchain", (w, h, b), lambda img=img, b=b: _fchain(img, b)))
            out.append(("separable", (w, h, b), lambda img=img, b=b: _separable(img, b)))
            out.append(("separable3", (w, h, b), lambda img=img, b=b: _separable(img, b, SEPARABLE3)))
            out.append(("morph", (w, h, b), lambda img=img, b=b: _morph(img, b)))
            out.append(("nonlinear", (w, h, b), lambda img=img, b=b: _nonlinear(img, b)))
            out.append(("laplace_float", (w, h, b), lambda img=img, b=b: _laplace_float(img, b)))
            out.append(("s16_local", (w, h, b), lambda img=img, b=b: _s16_local(img, b)))
            out.append(("edge_phase", (w, h, b), lambda img=img, b=b: _edge_phase(img, b, b)))
        for b0, b1 in ((BORDERS[0], BORDERS[2]), (BORDERS[4], BORDERS[1]), (BORDERS[3], BORDERS[4])):
            out.append(("mixed_borders", (w, h, b0, b1), lambda img=img, b0=b0, b1=b1: _mixed_borders(img, b0, b1)))
        for b in BORDERS[:3]:
            out.append(("uyvy", (w, h, b), lambda w=w, h=h, b=b: _uyvy(synth.uyvy_image(max(2, w // 2 * 2), h,
                                                                                        seed=7), b)))
    return out


CASES = _cases()


def _float_close(got, want, scale, rel=2e-6):
    err = np.abs(got.astype(np.float64) - want.astype(np.float64))
    assert (err <= rel * scale + 1e-6).all(), "max error %g" % (err / (scale + 1e-30)).max()


@pytest.mark.parametrize("case", range(len(CASES)), ids=["%s-%s" % (c[0], c[1]) for c in CASES])
def test_generated_equals_interpreter_and_oracle(ctx, case):
    name, shape, make = CASES[case]
    spec = make()
    log("codegen %s %s" % (name, shape))
    env = spec.run_oracle()
    gen, g1 = run_spec(spec, ctx, specialize=False)
    assert hvx.hvx_graph_query(g1, hvx.HVX_QUERY_NUM_GENERATED) >= 1
    ref, g0 = run_spec(spec, ctx, specialize=False, codegen=False)
    assert hvx.hvx_graph_query(g0, hvx.HVX_QUERY_NUM_GENERATED) == 0
    assert hvx.hvx_graph_query(g1, hvx.HVX_QUERY_NUM_KERNELS) == hvx.hvx_graph_query(g0, hvx.HVX_QUERY_NUM_KERNELS)
    valid = oracle.valid_masks(spec.oracle_graph(), spec.shapes())
    for out in spec.outputs:
        m = valid[out]
        a, b = gen[out], ref[out]
        if a.dtype == np.float32:
            assert np.array_equal(a.view(np.uint32)[m], b.view(np.uint32)[m]), "%s: generated != interpreter" % out
        else:
            assert np.array_equal(a[m], b[m]), "%s: generated != interpreter" % out
    float_outs = [o for o in spec.outputs if np.dtype(spec.outputs[o]) == np.float32]
    exact = gs.Spec(spec.nodes, spec.inputs, {o: d for o, d in spec.outputs.items() if o not in float_outs},
                    uyvy=spec.uyvy)
    if name == "tomasi":
        scale = np.abs(env["sxx"]) + np.abs(env["syy"]) + np.abs(env["sxy"])
        _float_close(gen["r"], env["r"], scale, 1e-5)
        amb = np.abs(env["r"] - 2e5) <= 1e-5 * scale + 1e-3
        assert not ((gen["out"] != env["out"]) & ~amb).any()
        return
    if name == "laplace_float":
        m = valid["f"]
        _float_close(gen["f"][m], env["f"][m], 1 + np.abs(env["f"][m]))
        amb = np.abs(env["f"] - 2.5) <= 1e-5 * (1 + np.abs(env["f"]))
        assert not ((gen["out"] != env["out"]) & ~amb & valid["out"]).any()
        exact = gs.Spec(spec.nodes, spec.inputs, {"lap": np.int16}, uyvy=spec.uyvy)
    compare(exact, gen, env, phase_names=("ph",))


@pytest.mark.parametrize("w,h", [(641, 363), (5, 3)])
def test_generated_reductions_fused(ctx, w, h):
    """Point and local producers fused into global operators (Table 2) in a
    generated kernel, against the interpreter and the oracle."""
    img = synth.edge_image(w, h, seed=5)
    spec = gs.Spec([gs.N("gaussian3x3", ["in"], ["g"]),
                    gs.N("histogram", ["g"], ["hist"], params={"bins": 32, "offset": 10, "range": 200}),
                    gs.N("min_max_loc", ["g"], ["mm"]),
                    gs.N("threshold", ["g"], ["out"], params={"thresh": 90})],
                   {"in": img}, {"out": np.uint8}, buffers={"hist": 32 * 4, "mm": 4128})
    log("codegen reductions %dx%d" % (w, h))
    gen, g1 = run_spec(spec, ctx, specialize=False)
    ref, g0 = run_spec(spec, ctx, specialize=False, codegen=False)
    assert hvx.hvx_graph_query(g1, hvx.HVX_QUERY_NUM_GENERATED) >= 1
    assert np.array_equal(gen["out"], ref["out"])
    assert np.array_equal(gen["hist"], ref["hist"])
    assert np.array_equal(gen["mm"][:16], ref["mm"][:16])
    env = spec.run_oracle()
    assert np.array_equal(gen["out"], env["out"])
    _check_buffers(spec, gen, env)
