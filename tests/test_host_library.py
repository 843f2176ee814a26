"""Host-side tests of libhvx.so: exports, handle checks, verification, dead
computation elimination and fusion planning.  No compute call is made, so
these run without a GPU (device pointers are never dereferenced before
process/schedule)."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import paper_2008_11476_amd as hvx
from tests import graphspec as gs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FAKE = 0x7f0000000000  # a 16-byte aligned address that is never dereferenced here


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(hvx.LIB_PATH):
        from paper_2008_11476_amd import build
        build.build()
    return hvx.lib()


@pytest.fixture
def ctx(lib):
    c = hvx.hvx_context_create(0)
    yield c
    hvx.hvx_context_release(c)


def _img(ctx, w, h, df, k=0):
    bpp = hvx.BYTES_PER_PIXEL[df]
    pitch = max(64, (w * bpp + 63) // 64 * 64)
    return hvx.hvx_image_from_ptr(ctx, w, h, df, FAKE + k * (1 << 28), pitch)


def test_exports_match_header(lib):
    hdr = open(os.path.join(ROOT, "include", "hvx.h")).read()
    declared = set(re.findall(r"\b(hvx_[a-z0-9_]+)\s*\(", hdr))
    out = subprocess.run(["nm", "-D", "--defined-only", hvx.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (hvx_[a-z0-9_]+)$", out, re.M))
    assert declared, "no declarations parsed"
    assert declared <= exported, "declared but not exported: %s" % sorted(declared - exported)
    for name in declared:
        assert hasattr(lib, name)


def test_status_names(lib):
    assert hvx.status_name(0) == "HVX_SUCCESS"
    assert hvx.status_name(-5) == "HVX_ERROR_INVALID_GRAPH"


def test_invalid_and_released_handles(ctx):
    g = hvx.hvx_graph_create(ctx)
    hvx.hvx_release_graph(g)
    with pytest.raises(hvx.HvxError) as e:
        hvx.hvx_graph_verify(g)
    assert e.value.status == hvx.HVX_ERROR_INVALID_REFERENCE
    with pytest.raises(hvx.HvxError) as e:
        hvx.hvx_graph_verify(12345678)
    assert e.value.status == hvx.HVX_ERROR_INVALID_REFERENCE
    # an image handle is not a graph handle
    a = _img(ctx, 8, 8, hvx.HVX_DF_U8)
    assert hvx.lib().hvx_graph_verify(a) == hvx.HVX_ERROR_INVALID_REFERENCE


def test_image_layout_checks(ctx):
    with pytest.raises(hvx.HvxError) as e:
        hvx.hvx_image_from_ptr(ctx, 100, 10, hvx.HVX_DF_U8, FAKE, 100)  # pitch not a multiple of 64
    assert e.value.status == hvx.HVX_ERROR_INVALID_PARAMETERS
    with pytest.raises(hvx.HvxError) as e:
        hvx.hvx_image_from_ptr(ctx, 100, 10, hvx.HVX_DF_S16, FAKE, 128)  # pitch < 2 * width
    assert e.value.status == hvx.HVX_ERROR_INVALID_PARAMETERS
    with pytest.raises(hvx.HvxError) as e:
        hvx.hvx_image_from_ptr(ctx, 7, 10, hvx.HVX_DF_UYVY, FAKE, 64)  # odd UYVY width
    assert e.value.status == hvx.HVX_ERROR_INVALID_DIMENSION
    with pytest.raises(hvx.HvxError) as e:
        hvx.hvx_image_from_ptr(ctx, 0, 10, hvx.HVX_DF_U8, FAKE, 64)
    assert e.value.status == hvx.HVX_ERROR_INVALID_DIMENSION


def _verify_status(g):
    return hvx.lib().hvx_graph_verify(g)


def test_verify_rejects_cycle_two_writers_and_formats(ctx):
    a = _img(ctx, 16, 16, hvx.HVX_DF_U8, 0)
    b = _img(ctx, 16, 16, hvx.HVX_DF_U8, 1)
    # cycle through virtual images
    g = hvx.hvx_graph_create(ctx)
    v1 = hvx.hvx_image_create_virtual(g)
    v2 = hvx.hvx_image_create_virtual(g)
    hvx.hvx_gaussian3x3_node(g, v1, v2)
    hvx.hvx_gaussian3x3_node(g, v2, v1)
    hvx.hvx_gaussian3x3_node(g, v2, b)
    assert _verify_status(g) == hvx.HVX_ERROR_INVALID_GRAPH
    # a node reading its own output
    g = hvx.hvx_graph_create(ctx)
    hvx.hvx_gaussian3x3_node(g, a, a)
    assert _verify_status(g) == hvx.HVX_ERROR_INVALID_GRAPH
    # two writers of one image
    g = hvx.hvx_graph_create(ctx)
    hvx.hvx_gaussian3x3_node(g, a, b)
    hvx.hvx_box3x3_node(g, a, b)
    assert _verify_status(g) == hvx.HVX_ERROR_INVALID_GRAPH
    # wrong formats and sizes
    s = _img(ctx, 16, 16, hvx.HVX_DF_S16, 2)
    g = hvx.hvx_graph_create(ctx)
    hvx.hvx_gaussian3x3_node(g, s, b)
    assert _verify_status(g) == hvx.HVX_ERROR_INVALID_FORMAT
    c = _img(ctx, 17, 16, hvx.HVX_DF_U8, 3)
    g = hvx.hvx_graph_create(ctx)
    hvx.hvx_gaussian3x3_node(g, a, c)
    assert _verify_status(g) == hvx.HVX_ERROR_INVALID_DIMENSION
    g = hvx.hvx_graph_create(ctx)
    hvx.hvx_magnitude_node(g, s, _img(ctx, 17, 16, hvx.HVX_DF_S16, 4), _img(ctx, 16, 16, hvx.HVX_DF_S16, 5))
    assert _verify_status(g) == hvx.HVX_ERROR_INVALID_DIMENSION
    # a virtual image read but never written
    g = hvx.hvx_graph_create(ctx)
    hvx.hvx_gaussian3x3_node(g, hvx.hvx_image_create_virtual(g), b)
    assert _verify_status(g) == hvx.HVX_ERROR_INVALID_GRAPH
    # a virtual image of another graph
    g0 = hvx.hvx_graph_create(ctx)
    foreign = hvx.hvx_image_create_virtual(g0)
    g = hvx.hvx_graph_create(ctx)
    hvx.hvx_gaussian3x3_node(g, a, foreign)
    hvx.hvx_gaussian3x3_node(g, foreign, b)
    assert _verify_status(g) == hvx.HVX_ERROR_INVALID_GRAPH
    # an empty graph
    assert _verify_status(hvx.hvx_graph_create(ctx)) == hvx.HVX_ERROR_INVALID_GRAPH


def test_virtual_declared_format_mismatch(ctx):
    a = _img(ctx, 16, 16, hvx.HVX_DF_U8, 0)
    b = _img(ctx, 16, 16, hvx.HVX_DF_U8, 1)
    g = hvx.hvx_graph_create(ctx)
    v = hvx.hvx_image_create_virtual(g, 0, 0, hvx.HVX_DF_S16)
    hvx.hvx_gaussian3x3_node(g, a, v)
    hvx.hvx_gaussian3x3_node(g, v, b)
    assert _verify_status(g) == hvx.HVX_ERROR_INVALID_FORMAT


def _golden_dce():
    rows = []
    for line in open(os.path.join(ROOT, "tests", "golden", "listing1_dce.txt")):
        line = line.strip()
        if line and not line.startswith("#"):
            name, state = line.split()
            rows.append((name, state == "live"))
    return rows


def test_listing1_dead_computation_elimination(ctx):
    """The gx output of the Sobel node in the Section 3.1 example is dead."""
    w, h = 64, 32
    frame = np.zeros((h, 2 * w), np.uint8)
    spec = gs.listing1_spec(frame)
    imgs = {"in": _img(ctx, w, h, hvx.HVX_DF_UYVY, 0), "out": _img(ctx, w, h, hvx.HVX_DF_U8, 1)}
    g, _, _ = gs.build_hvx(spec, ctx, imgs)
    hvx.hvx_graph_verify(g)
    expect = _golden_dce()
    assert hvx.hvx_graph_query(g, hvx.HVX_QUERY_NUM_NODES) == 5
    assert hvx.hvx_graph_query(g, hvx.HVX_QUERY_NUM_OPS) == len(expect)
    assert hvx.hvx_graph_query(g, hvx.HVX_QUERY_NUM_LIVE_OPS) == sum(live for _, live in expect)
    mask = hvx.hvx_graph_query(g, hvx.HVX_QUERY_OP_LIVE_MASK)
    assert [bool(mask >> i & 1) for i in range(len(expect))] == [live for _, live in expect]
    # fused into one kernel; only the UYVY input and the U8 output touch memory
    assert hvx.hvx_graph_query(g, hvx.HVX_QUERY_NUM_KERNELS) == 1
    assert hvx.hvx_graph_query(g, hvx.HVX_QUERY_ALG_BYTES) == w * h * 3
    # DCE off: all six operators stay
    hvx.hvx_graph_set_option(g, hvx.HVX_OPT_DCE, 0)
    hvx.hvx_graph_verify(g)
    assert hvx.hvx_graph_query(g, hvx.HVX_QUERY_NUM_LIVE_OPS) == len(expect)
    # fusion off: one kernel per live operator, intermediates materialised
    hvx.hvx_graph_set_option(g, hvx.HVX_OPT_DCE, 1)
    hvx.hvx_graph_set_option(g, hvx.HVX_OPT_FUSION, 0)
    hvx.hvx_graph_verify(g)
    assert hvx.hvx_graph_query(g, hvx.HVX_QUERY_NUM_KERNELS) == 5
    assert hvx.hvx_graph_query(g, hvx.HVX_QUERY_SCRATCH_BYTES) > 0


def test_dce_algorithm1_cases(ctx):
    """Algorithm 1 on hand-built graphs: an intermediate non-virtual image is
    both an input and a result; a virtual branch reaching no non-virtual image
    is dead; an isolated non-virtual image is harmless."""
    a = _img(ctx, 32, 32, hvx.HVX_DF_U8, 0)
    mid = _img(ctx, 32, 32, hvx.HVX_DF_U8, 1)
    out = _img(ctx, 32, 32, hvx.HVX_DF_U8, 2)
    _img(ctx, 32, 32, hvx.HVX_DF_U8, 3)  # isolated
    g = hvx.hvx_graph_create(ctx)
    hvx.hvx_gaussian3x3_node(g, a, mid)                 # op 0: live (non-virtual result)
    hvx.hvx_box3x3_node(g, mid, out)                    # op 1: live
    dead = hvx.hvx_image_create_virtual(g)
    hvx.hvx_gaussian5x5_node(g, mid, dead)              # op 2: dead (virtual, unread)
    dead2 = hvx.hvx_image_create_virtual(g)
    hvx.hvx_box3x3_node(g, dead, dead2)                 # op 3: dead
    hvx.hvx_graph_verify(g)
    assert hvx.hvx_graph_query(g, hvx.HVX_QUERY_OP_LIVE_MASK) == 0b0011
    assert hvx.hvx_graph_query(g, hvx.HVX_QUERY_NUM_LIVE_OPS) == 2


def test_sobel_lowering_and_kernel_choice(ctx):
    w, h = 256, 64
    img = np.zeros((h, w), np.uint8)
    for spec, kind, nops in ((gs.edge_spec(img), 1, 5), (gs.edge_spec(img, phase=True), 1, 6),
                             (gs.corner_spec(img), 2, 10), (gs.gauss5_spec(img), 3, 1)):
        imgs = {"in": _img(ctx, w, h, hvx.HVX_DF_U8, 0)}
        for i, name in enumerate(spec.outputs):
            imgs[name] = _img(ctx, w, h, hvx.HVX_DF_U8, 1 + i)
        g, _, _ = gs.build_hvx(spec, ctx, imgs)
        hvx.hvx_graph_verify(g)
        assert hvx.hvx_graph_query(g, hvx.HVX_QUERY_NUM_LIVE_OPS) == nops
        assert hvx.hvx_graph_query(g, hvx.HVX_QUERY_NUM_KERNELS) == 1
        expected_kind = kind if kind != 2 else hvx.hvx_graph_query(g, hvx.HVX_QUERY_KERNEL_KIND)
        assert hvx.hvx_graph_query(g, hvx.HVX_QUERY_KERNEL_KIND) == expected_kind
        assert hvx.hvx_graph_query(g, hvx.HVX_QUERY_ALG_BYTES) == w * h * (1 + len(spec.outputs))
        hvx.hvx_graph_set_option(g, hvx.HVX_OPT_SPECIALIZE, 0)
        hvx.hvx_graph_verify(g)
        assert hvx.hvx_graph_query(g, hvx.HVX_QUERY_KERNEL_KIND) == 0
        assert hvx.hvx_graph_query(g, hvx.HVX_QUERY_NUM_KERNELS) == 1


def test_unfused_edge_graph_bytes(ctx):
    """Node-by-node execution of the lowered edge graph moves 17 B/px
    (Gaussian r1 w1, the two Sobel operators r1 w2 each, Magnitude r4 w2,
    Threshold r2 w1); fused, 2 B/px."""
    w, h = 128, 32
    spec = gs.edge_spec(np.zeros((h, w), np.uint8))
    g, _, _ = gs.build_hvx(spec, ctx, {"in": _img(ctx, w, h, hvx.HVX_DF_U8, 0),
                                       "out": _img(ctx, w, h, hvx.HVX_DF_U8, 1)})
    hvx.hvx_graph_set_option(g, hvx.HVX_OPT_FUSION, 0)
    hvx.hvx_graph_verify(g)
    assert hvx.hvx_graph_query(g, hvx.HVX_QUERY_NUM_KERNELS) == 5
    assert hvx.hvx_graph_query(g, hvx.HVX_QUERY_HBM_BYTES) == 17 * w * h
    hvx.hvx_graph_set_option(g, hvx.HVX_OPT_FUSION, 1)
    hvx.hvx_graph_verify(g)
    assert hvx.hvx_graph_query(g, hvx.HVX_QUERY_HBM_BYTES) == 2 * w * h


def test_graph_edit_unverifies(ctx):
    a = _img(ctx, 16, 16, hvx.HVX_DF_U8, 0)
    b = _img(ctx, 16, 16, hvx.HVX_DF_U8, 1)
    g = hvx.hvx_graph_create(ctx)
    n = hvx.hvx_gaussian3x3_node(g, a, b)
    hvx.hvx_graph_verify(g)
    assert hvx.hvx_graph_query(g, hvx.HVX_QUERY_NUM_LIVE_OPS) == 1
    hvx.hvx_node_set_border(n, hvx.HVX_BORDER_CONSTANT, 7)
    with pytest.raises(hvx.HvxError) as e:
        hvx.hvx_graph_query(g, hvx.HVX_QUERY_NUM_LIVE_OPS)
    assert e.value.status == hvx.HVX_ERROR_NOT_VERIFIED


def test_release_semantics(ctx):
    a = _img(ctx, 16, 16, hvx.HVX_DF_U8, 0)
    b = _img(ctx, 16, 16, hvx.HVX_DF_U8, 1)
    g = hvx.hvx_graph_create(ctx)
    n = hvx.hvx_gaussian3x3_node(g, a, b)
    hvx.hvx_release_node(n)      # the node stays in the graph
    hvx.hvx_release_image(a)     # still used: handle retired, object kept
    with pytest.raises(hvx.HvxError):
        hvx.hvx_image_query(a)
    hvx.hvx_graph_verify(g)
    assert hvx.hvx_graph_query(g, hvx.HVX_QUERY_NUM_LIVE_OPS) == 1


def test_convolution_checks(ctx):
    with pytest.raises(hvx.HvxError) as e:
        hvx.hvx_convolution_create(ctx, np.ones((3, 3)), 3)
    assert e.value.status == hvx.HVX_ERROR_INVALID_PARAMETERS
    with pytest.raises(hvx.HvxError) as e:
        hvx.hvx_convolution_create(ctx, np.ones((2, 3)), 1)
    assert e.value.status == hvx.HVX_ERROR_INVALID_DIMENSION
    c = hvx.hvx_convolution_create(ctx, np.ones((3, 5)), 16)
    hvx.hvx_release_convolution(c)


def test_no_device_errors_cleanly(ctx):
    """Without a GPU, device work reports HVX_ERROR_DEVICE (never a crash)."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    a = _img(ctx, 16, 16, hvx.HVX_DF_U8, 0)
    b = _img(ctx, 16, 16, hvx.HVX_DF_U8, 1)
    g = hvx.hvx_graph_create(ctx)
    hvx.hvx_gaussian3x3_node(g, a, b)
    assert hvx.lib().hvx_graph_process(g) == hvx.HVX_ERROR_DEVICE


def test_global_ops_reject_2_31_pixels(ctx):
    """The global operators count in 32 bits: an image of 2^31 pixels or more
    (which the image constructors accept) is refused before any device work,
    so a constant 65536x65536 image can never wrap a bin or a count."""
    import torch
    big = _img(ctx, 65536, 32768, hvx.HVX_DF_U8, 0)      # exactly 2^31 pixels
    big16 = _img(ctx, 65536, 65536, hvx.HVX_DF_S16, 1)
    L = hvx.lib()
    buf = ctypes.c_void_p(FAKE)
    assert L.hvx_histogram(ctx, big, 256, 0, 256, buf, None) == hvx.HVX_ERROR_INVALID_DIMENSION
    assert L.hvx_min_max(ctx, big16, buf, None) == hvx.HVX_ERROR_INVALID_DIMENSION
    assert L.hvx_min_max_count(ctx, big, buf, None) == hvx.HVX_ERROR_INVALID_DIMENSION
    assert L.hvx_min_max_loc(ctx, big16, buf, buf, buf, 16, None) == hvx.HVX_ERROR_INVALID_DIMENSION
    assert L.hvx_equalize_hist(ctx, big, big, buf, None) == hvx.HVX_ERROR_INVALID_DIMENSION
    assert L.hvx_mean_std_dev(ctx, big, buf, None) == hvx.HVX_ERROR_INVALID_DIMENSION
    assert "2^31" in hvx.hvx_last_error(ctx)
    if not torch.cuda.is_available():
        # one pixel fewer passes the size check and only then needs the device
        ok = _img(ctx, 65535, 32768, hvx.HVX_DF_U8, 2)
        assert L.hvx_min_max(ctx, ok, buf, None) == hvx.HVX_ERROR_DEVICE


def test_tune_cache_roundtrip(ctx, tmp_path):
    p = tmp_path / "tune.json"
    p.write_text('{\n  "gfx950|k1:3840x2160:3.2.0,": [32, 1, 12.5]\n}\n')
    hvx.hvx_context_load_tune_cache(ctx, str(p))
    q = tmp_path / "out.json"
    hvx.hvx_context_save_tune_cache(ctx, str(q))
    assert '"gfx950|k1:3840x2160:3.2.0,": [32, 1, 12.5]' in q.read_text()


def test_tune_cache_plan_choice_roundtrip(ctx, tmp_path):
    """A plan choice (cut values and generated tiles) survives a save and a
    load; malformed plan lists are refused."""
    p = tmp_path / "tune.json"
    key = "plan|f1.s1.c1:2.2(0,-1,-1>1)20.2(0,1,-1>2)|1.64x48,1.64x48v,2.64x48,"
    p.write_text('{\n  "%s": [0, 1, 7.25, [1, 5], [[0, 64, 32], [3, 128, 8]]]\n}\n' % key)
    hvx.hvx_context_load_tune_cache(ctx, str(p))
    q = tmp_path / "out.json"
    hvx.hvx_context_save_tune_cache(ctx, str(q))
    assert '"%s": [0, 1, 7.25, [1, 5], [[0, 64, 32], [3, 128, 8]]]' % key in q.read_text()
    bad = tmp_path / "bad.json"
    bad.write_text('{"plan|x": [0, 1, 2.0, [1], [[0, 64]]]}')
    with pytest.raises(hvx.HvxError):
        hvx.hvx_context_load_tune_cache(ctx, str(bad))


EXPR_CORPUS = ["a", "a + b * c", "-a - -b", "(a + 1) * (b - 2) / 3", "min(a, b)", "max(a, min(b, c))", "abs(a)",
               "clamp(a, 0, 9)", "gt(a, b)", "sel(a, b, c)", "a / 0", "2147483647 + a", "sqrt(a)", "a * 0.5",
               "a +", "a b", "(a", "a)", "min(a)", "max(a, b, c)", "foo(a)", "d", "a ** 2", "a % 2", "a // 2",
               "a > b", "", "   ", "1e3", "a[1, 0]", "a[-2, 2] + a", "a[3, 0]", "a[1]", "b[0, 0]", "a[1, 0",
               "a[ -1 , 1 ] * 2", "a[1.0, 0]", "2147483648", "-2147483648 + a", "clamp(a, b)", "sel(a, b)"]


@pytest.mark.parametrize("local", [False, True])
def test_user_kernel_parser_agrees_with_the_oracle_grammar(ctx, local):
    """The library's parser (node creation plus verification of an integer
    kernel) accepts exactly the expressions the oracle's own parser accepts."""
    from oracle import custom
    for expr in EXPR_CORPUS:
        try:
            custom.check(expr, 1 if local else 3, False, local=local)
            want = True
        except ValueError:
            want = False
        ims = [_img(ctx, 16, 4, hvx.HVX_DF_U8, k) for k in range(3)] + [_img(ctx, 16, 4, hvx.HVX_DF_S16, 3)]
        g = hvx.hvx_graph_create(ctx)
        try:
            if local:
                hvx.hvx_custom_local_node(g, expr, ims[0], hvx.HVX_DF_S16, ims[3], ctx=ctx)
            else:
                hvx.hvx_custom_point_node(g, expr, ims[:3], hvx.HVX_DF_S16, ims[3], ctx=ctx)
            got = _verify_status(g) == hvx.HVX_SUCCESS
        except hvx.HvxError:
            got = False
        hvx.hvx_release_graph(g)
        for im in ims:
            hvx.hvx_release_image(im)
        assert got == want, (expr, local, got, want)
