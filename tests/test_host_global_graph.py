"""Host-side tests of global operators as graph nodes (Table 2): buffer
objects, argument checks, verification errors, dead-computation elimination
and the planning of phases and fused reductions.  No compute call is made,
so these run without a GPU (device pointers are never dereferenced before
process/schedule)."""
import pytest

import paper_2008_11476_amd as hvx

FAKE = 0x7f0000000000  # 16-byte aligned, never dereferenced here


@pytest.fixture(scope="module")
def lib():
    import os
    if not os.path.exists(hvx.LIB_PATH):
        from paper_2008_11476_amd import build
        build.build()
    return hvx.lib()


@pytest.fixture
def ctx(lib):
    c = hvx.hvx_context_create(0)
    yield c
    hvx.hvx_context_release(c)


def _img(ctx, w, h, df=hvx.HVX_DF_U8, k=0):
    bpp = hvx.BYTES_PER_PIXEL[df]
    pitch = max(64, (w * bpp + 63) // 64 * 64)
    return hvx.hvx_image_from_ptr(ctx, w, h, df, FAKE + k * (1 << 28), pitch)


def _buf(ctx, nbytes, k=0):
    return hvx.hvx_buffer_from_ptr(ctx, FAKE + (1 << 40) + k * (1 << 20), nbytes)


def _status(fn, *a, **kw):
    try:
        fn(*a, **kw)
    except hvx.HvxError as e:
        return e.status
    return 0


def _q(g, attr):
    return hvx.hvx_graph_query(g, attr)


def test_buffer_argument_checks(ctx):
    assert _status(hvx.hvx_buffer_from_ptr, ctx, 0, 64) == hvx.HVX_ERROR_INVALID_PARAMETERS
    assert _status(hvx.hvx_buffer_from_ptr, ctx, FAKE + 4, 64) == hvx.HVX_ERROR_INVALID_PARAMETERS
    assert _status(hvx.hvx_buffer_from_ptr, ctx, FAKE, 0) == hvx.HVX_ERROR_INVALID_DIMENSION
    b = _buf(ctx, 64)
    hvx.hvx_release_buffer(b)
    assert _status(hvx.hvx_release_buffer, b) == hvx.HVX_ERROR_INVALID_REFERENCE


def test_global_node_argument_checks(ctx):
    g = hvx.hvx_graph_create(ctx)
    a, b = _img(ctx, 64, 32), _buf(ctx, 1024)
    for bins, off, rng in [(0, 0, 256), (257, 0, 256), (10, 0, 5), (16, 200, 100)]:
        assert _status(hvx.hvx_histogram_node, g, a, bins, off, rng, b) == hvx.HVX_ERROR_INVALID_PARAMETERS
    # a buffer is not an image, an image is not a buffer
    assert _status(hvx.hvx_min_max_node, g, b, b) == hvx.HVX_ERROR_INVALID_REFERENCE
    assert _status(hvx.hvx_min_max_node, g, a, a) == hvx.HVX_ERROR_INVALID_REFERENCE
    assert _status(hvx.hvx_gaussian3x3_node, g, a, b) == hvx.HVX_ERROR_INVALID_REFERENCE
    # locations and a capacity go together
    assert _status(hvx.hvx_min_max_loc_node, g, a, b, None, 4) == hvx.HVX_ERROR_INVALID_PARAMETERS
    assert _status(hvx.hvx_min_max_loc_node, g, a, b, _buf(ctx, 64, 1), 0) == hvx.HVX_ERROR_INVALID_PARAMETERS


@pytest.mark.parametrize("make,need", [
    (lambda g, a, b: hvx.hvx_histogram_node(g, a, 16, 0, 256, b), 64),
    (lambda g, a, b: hvx.hvx_min_max_node(g, a, b), 8),
    (lambda g, a, b: hvx.hvx_min_max_loc_node(g, a, b, None, 0), 4128),
    (lambda g, a, b: hvx.hvx_mean_std_dev_node(g, a, b), 24),
])
def test_verify_checks_result_buffer_size(ctx, make, need):
    for nbytes, want in [(need - 4, hvx.HVX_ERROR_INVALID_DIMENSION), (need, 0)]:
        g = hvx.hvx_graph_create(ctx)
        make(g, _img(ctx, 100, 50), _buf(ctx, nbytes))
        assert _status(hvx.hvx_graph_verify, g) == want, (need, nbytes)


def test_verify_checks_location_buffer_size(ctx):
    for nbytes, want in [(16 * 10 - 1, hvx.HVX_ERROR_INVALID_DIMENSION), (16 * 10, 0)]:
        g = hvx.hvx_graph_create(ctx)
        hvx.hvx_min_max_loc_node(g, _img(ctx, 100, 50), _buf(ctx, 4128), _buf(ctx, nbytes, 1), 10)
        assert _status(hvx.hvx_graph_verify, g) == want


def test_verify_checks_global_input_formats(ctx):
    s16 = _img(ctx, 64, 8, hvx.HVX_DF_S16)
    f32 = _img(ctx, 64, 8, hvx.HVX_DF_F32, 1)
    for make in (lambda g: hvx.hvx_histogram_node(g, s16, 256, 0, 256, _buf(ctx, 1024)),
                 lambda g: hvx.hvx_mean_std_dev_node(g, s16, _buf(ctx, 64)),
                 lambda g: hvx.hvx_min_max_node(g, f32, _buf(ctx, 64)),
                 lambda g: hvx.hvx_equalize_hist_node(g, s16, _img(ctx, 64, 8, hvx.HVX_DF_U8, 2))):
        g = hvx.hvx_graph_create(ctx)
        make(g)
        assert _status(hvx.hvx_graph_verify, g) == hvx.HVX_ERROR_INVALID_FORMAT
    # S16 is accepted by min/max and MinMaxLoc
    g = hvx.hvx_graph_create(ctx)
    hvx.hvx_min_max_loc_node(g, s16, _buf(ctx, 4128), None, 0)
    hvx.hvx_graph_verify(g)


def test_two_writers_of_one_buffer(ctx):
    g = hvx.hvx_graph_create(ctx)
    a, b = _img(ctx, 64, 8), _buf(ctx, 64)
    hvx.hvx_min_max_node(g, a, b)
    hvx.hvx_mean_std_dev_node(g, a, b)
    assert _status(hvx.hvx_graph_verify, g) == hvx.HVX_ERROR_INVALID_GRAPH


def test_lone_global_operator_uses_the_streaming_kernel(ctx):
    g = hvx.hvx_graph_create(ctx)
    hvx.hvx_histogram_node(g, _img(ctx, 640, 480), 256, 0, 256, _buf(ctx, 1024))
    hvx.hvx_graph_verify(g)
    assert _q(g, hvx.HVX_QUERY_NUM_KERNELS) == 1
    assert _q(g, hvx.HVX_QUERY_KERNEL_KIND) == 4


def test_producer_fused_into_the_reduction(ctx):
    # Gaussian3x3 -> histogram of the (virtual) result: one kernel, nothing materialised
    g = hvx.hvx_graph_create(ctx)
    v = hvx.hvx_image_create_virtual(g)
    hvx.hvx_gaussian3x3_node(g, _img(ctx, 640, 480), v)
    hvx.hvx_histogram_node(g, v, 256, 0, 256, _buf(ctx, 1024))
    hvx.hvx_graph_verify(g)
    assert _q(g, hvx.HVX_QUERY_NUM_KERNELS) == 1
    assert _q(g, hvx.HVX_QUERY_KERNEL_KIND) == 0
    assert _q(g, hvx.HVX_QUERY_SCRATCH_BYTES) == 0
    # bytes moved: the input image and the counts only
    assert _q(g, hvx.HVX_QUERY_HBM_BYTES) == 640 * 480 + 1024


def test_image_output_and_reductions_in_one_kernel(ctx):
    g = hvx.hvx_graph_create(ctx)
    a, o = _img(ctx, 640, 480), _img(ctx, 640, 480, k=1)
    hvx.hvx_gaussian3x3_node(g, a, o)
    hvx.hvx_min_max_node(g, o, _buf(ctx, 64))
    hvx.hvx_mean_std_dev_node(g, o, _buf(ctx, 64, 1))
    hvx.hvx_graph_verify(g)
    assert _q(g, hvx.HVX_QUERY_NUM_KERNELS) == 1


def test_three_reductions_split_into_operators(ctx):
    g = hvx.hvx_graph_create(ctx)
    v = hvx.hvx_image_create_virtual(g)
    hvx.hvx_gaussian3x3_node(g, _img(ctx, 640, 480), v)
    hvx.hvx_min_max_node(g, v, _buf(ctx, 64))
    hvx.hvx_mean_std_dev_node(g, v, _buf(ctx, 64, 1))
    hvx.hvx_histogram_node(g, v, 8, 0, 256, _buf(ctx, 64, 2))
    hvx.hvx_graph_verify(g)
    # one kernel holds at most two reductions: node by node instead
    assert _q(g, hvx.HVX_QUERY_NUM_KERNELS) == 4
    assert _q(g, hvx.HVX_QUERY_SCRATCH_BYTES) == 640 * 480


def test_phases_order_the_equalize_hist_kernels(ctx):
    # EqualizeHist -> Gaussian: histogram + mapping first, then the mapping
    # applied and the Gaussian fused in one later kernel
    g = hvx.hvx_graph_create(ctx)
    v = hvx.hvx_image_create_virtual(g)
    hvx.hvx_equalize_hist_node(g, _img(ctx, 640, 480), v)
    hvx.hvx_gaussian3x3_node(g, v, _img(ctx, 640, 480, k=1))
    hvx.hvx_graph_verify(g)
    assert _q(g, hvx.HVX_QUERY_NUM_OPS) == 3
    assert _q(g, hvx.HVX_QUERY_NUM_KERNELS) == 2
    assert _q(g, hvx.HVX_QUERY_KERNEL_KIND) == 4
    assert _q(g, hvx.HVX_QUERY_SCRATCH_BYTES) == 1280  # the counts and the table
    # Gaussian -> EqualizeHist: the Gaussian fused into the histogram; the
    # mapping, applied later, needs the Gaussian again: materialised
    g = hvx.hvx_graph_create(ctx)
    v = hvx.hvx_image_create_virtual(g)
    hvx.hvx_gaussian3x3_node(g, _img(ctx, 640, 480), v)
    hvx.hvx_equalize_hist_node(g, v, _img(ctx, 640, 480, k=1))
    hvx.hvx_graph_verify(g)
    assert _q(g, hvx.HVX_QUERY_NUM_KERNELS) == 2
    assert _q(g, hvx.HVX_QUERY_KERNEL_KIND) == 0
    assert _q(g, hvx.HVX_QUERY_SCRATCH_BYTES) == 640 * 480 + 1280


def test_min_max_loc_lowering(ctx):
    # counts alone: one operator; with locations a second, in a later kernel
    g = hvx.hvx_graph_create(ctx)
    hvx.hvx_min_max_loc_node(g, _img(ctx, 64, 32), _buf(ctx, 4128), None, 0)
    hvx.hvx_graph_verify(g)
    assert _q(g, hvx.HVX_QUERY_NUM_OPS) == 1
    g = hvx.hvx_graph_create(ctx)
    v = hvx.hvx_image_create_virtual(g)
    hvx.hvx_gaussian5x5_node(g, _img(ctx, 640, 480), v)
    hvx.hvx_min_max_loc_node(g, v, _buf(ctx, 4128), _buf(ctx, 16 * 8, 1), 8)
    hvx.hvx_graph_verify(g)
    assert _q(g, hvx.HVX_QUERY_NUM_OPS) == 3
    assert _q(g, hvx.HVX_QUERY_NUM_KERNELS) == 2  # Gaussian + counts, then the location pass
    assert _q(g, hvx.HVX_QUERY_SCRATCH_BYTES) == 640 * 480


def test_dead_code_elimination_keeps_reduced_chains(ctx):
    # Gaussian -> {histogram, Sobel -> (virtual, unread)}: the Sobel is dead,
    # the Gaussian lives because its values reach a result buffer
    g = hvx.hvx_graph_create(ctx)
    v, gx = hvx.hvx_image_create_virtual(g), hvx.hvx_image_create_virtual(g)
    hvx.hvx_gaussian3x3_node(g, _img(ctx, 320, 240), v)
    hvx.hvx_sobel3x3_node(g, v, gx, None)
    hvx.hvx_histogram_node(g, v, 4, 0, 256, _buf(ctx, 64))
    hvx.hvx_graph_verify(g)
    assert _q(g, hvx.HVX_QUERY_NUM_OPS) == 3
    assert _q(g, hvx.HVX_QUERY_NUM_LIVE_OPS) == 2
    assert _q(g, hvx.HVX_QUERY_OP_LIVE_MASK) == 0b101
    assert _q(g, hvx.HVX_QUERY_NUM_KERNELS) == 1


def test_fusion_off_runs_node_by_node(ctx):
    g = hvx.hvx_graph_create(ctx)
    v = hvx.hvx_image_create_virtual(g)
    hvx.hvx_gaussian3x3_node(g, _img(ctx, 640, 480), v)
    hvx.hvx_histogram_node(g, v, 256, 0, 256, _buf(ctx, 1024))
    hvx.hvx_graph_set_option(g, hvx.HVX_OPT_FUSION, 0)
    hvx.hvx_graph_verify(g)
    assert _q(g, hvx.HVX_QUERY_NUM_KERNELS) == 2
    assert _q(g, hvx.HVX_QUERY_SCRATCH_BYTES) == 640 * 480


def test_global_nodes_refuse_images_of_2_31_pixels(ctx):
    """The counts of a global operator are 32-bit: verification refuses an
    input of 2^31 pixels or more, and takes one pixel fewer."""
    for h, want in ((32768, hvx.HVX_ERROR_INVALID_DIMENSION), (32767, 0)):
        g = hvx.hvx_graph_create(ctx)
        a = _img(ctx, 65536, h)
        hvx.hvx_histogram_node(g, a, 16, 0, 256, _buf(ctx, 64))
        assert _status(hvx.hvx_graph_verify, g) == want
        if want:
            assert "2^31" in hvx.hvx_last_error(ctx)
        hvx.hvx_release_graph(g)
