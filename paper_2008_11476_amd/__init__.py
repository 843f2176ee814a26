"""hvx: OpenVX-style image graphs as fused HIP kernels on gfx950.

Thin ctypes binding over ``libhvx.so``: the functions below carry the names of
the C ABI in ``include/hvx.h`` and only marshal arguments; every step of graph
execution runs in the library's HIP kernels.  Output parameters of the C
calls are returned; a non-zero status raises :class:`HvxError` with the
library's message.  PyTorch is used only for device memory and streams
(see :func:`alloc_image`, :func:`tensor_args`).
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhvx.so")

# ---- constants (include/hvx.h) ---------------------------------------------
HVX_SUCCESS = 0
HVX_ERROR_INVALID_REFERENCE = -1
HVX_ERROR_INVALID_PARAMETERS = -2
HVX_ERROR_INVALID_FORMAT = -3
HVX_ERROR_INVALID_DIMENSION = -4
HVX_ERROR_INVALID_GRAPH = -5
HVX_ERROR_NOT_VERIFIED = -6
HVX_ERROR_NO_MEMORY = -7
HVX_ERROR_NOT_SUPPORTED = -8
HVX_ERROR_DEVICE = -9

HVX_DF_VIRT, HVX_DF_U8, HVX_DF_S16, HVX_DF_S32, HVX_DF_F32, HVX_DF_UYVY = range(6)
HVX_BORDER_UNDEFINED, HVX_BORDER_CONSTANT, HVX_BORDER_REPLICATE, HVX_BORDER_MIRROR, HVX_BORDER_REPEAT = range(5)
HVX_POLICY_SATURATE, HVX_POLICY_WRAP = 0, 1
HVX_CHANNEL_Y = 0
HVX_OPT_FUSION, HVX_OPT_DCE, HVX_OPT_TILE, HVX_OPT_SPECIALIZE, HVX_OPT_XCD_REMAP, HVX_OPT_CODEGEN = 1, 2, 3, 4, 5, 6
(HVX_QUERY_NUM_NODES, HVX_QUERY_NUM_OPS, HVX_QUERY_NUM_LIVE_OPS, HVX_QUERY_NUM_KERNELS, HVX_QUERY_ALG_BYTES,
 HVX_QUERY_HBM_BYTES, HVX_QUERY_KERNEL_KIND, HVX_QUERY_SCRATCH_BYTES, HVX_QUERY_OP_LIVE_MASK,
 HVX_QUERY_ROWS_PER_ITEM, HVX_QUERY_NUM_GENERATED, HVX_QUERY_PLAN_CUTS, HVX_QUERY_GEN_TILE) = range(1, 14)
HVX_SERVER_CONTINUOUS, HVX_SERVER_PLAIN = 0, 1
HVX_BATCH_PERSISTENT, HVX_BATCH_USE_GRAPH, HVX_BATCH_ROWS = 1, 2, 3

BYTES_PER_PIXEL = {HVX_DF_U8: 1, HVX_DF_S16: 2, HVX_DF_S32: 4, HVX_DF_F32: 4, HVX_DF_UYVY: 2}


HVX_MEMORY_HOST, HVX_MEMORY_DEVICE = 0, 1


class hvx_binding(ctypes.Structure):
    """One image of a served request (include/hvx.h): the template image it
    stands for, the request's pixels and their row pitch."""
    _fields_ = [("image", ctypes.c_void_p), ("ptr", ctypes.c_void_p), ("pitch", ctypes.c_size_t)]


class HvxError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("%s: %s" % (status_name(status) if _lib else status, message))
        self.status = status


_lib = None
_vp = ctypes.c_void_p
_P = ctypes.POINTER


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libhvx.so is not built (%s); run `python -m paper_2008_11476_amd.build`" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    sig = {
        "hvx_context_create": [ctypes.c_int, _P(_vp)],
        "hvx_context_release": [_P(_vp)],
        "hvx_image_from_ptr": [_vp, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int, _vp, ctypes.c_size_t, _P(_vp)],
        "hvx_image_create": [_vp, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int, _P(_vp)],
        "hvx_image_swap_ptr": [_vp, _vp, ctypes.c_size_t],
        "hvx_image_query": [_vp, _P(ctypes.c_uint32), _P(ctypes.c_uint32), _P(ctypes.c_int), _P(_vp),
                            _P(ctypes.c_size_t)],
        "hvx_image_copy": [_vp, _vp, ctypes.c_size_t, ctypes.c_int],
        "hvx_image_create_virtual": [_vp, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int, _P(_vp)],
        "hvx_convolution_create": [_vp, ctypes.c_uint32, ctypes.c_uint32, _P(ctypes.c_int16), ctypes.c_uint32,
                                   _P(_vp)],
        "hvx_graph_create": [_vp, _P(_vp)],
        "hvx_channel_extract_node": [_vp, _vp, ctypes.c_int, _vp, _P(_vp)],
        "hvx_gaussian3x3_node": [_vp, _vp, _vp, _P(_vp)],
        "hvx_gaussian5x5_node": [_vp, _vp, _vp, _P(_vp)],
        "hvx_box3x3_node": [_vp, _vp, _vp, _P(_vp)],
        "hvx_dilate3x3_node": [_vp, _vp, _vp, _P(_vp)],
        "hvx_erode3x3_node": [_vp, _vp, _vp, _P(_vp)],
        "hvx_median3x3_node": [_vp, _vp, _vp, _P(_vp)],
        "hvx_nonlinear_filter_node": [_vp, ctypes.c_int, _vp, ctypes.c_uint32, ctypes.c_uint32, _vp, _vp, _P(_vp)],
        "hvx_non_max_suppression_node": [_vp, _vp, ctypes.c_uint32, _vp, _P(_vp)],
        "hvx_custom_point_node": [_vp, ctypes.c_char_p, _P(_vp), ctypes.c_uint32, ctypes.c_int, _vp, _P(_vp)],
        "hvx_custom_local_node": [_vp, ctypes.c_char_p, _vp, ctypes.c_int, _vp, _P(_vp)],
        "hvx_histogram": [_vp, _vp, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, _vp, _vp],
        "hvx_min_max": [_vp, _vp, _vp, _vp],
        "hvx_mean_std_dev": [_vp, _vp, _vp, _vp],
        "hvx_min_max_count": [_vp, _vp, _vp, _vp],
        "hvx_equalize_hist": [_vp, _vp, _vp, _vp, _vp],
        "hvx_equalize_hist_noalloc": [_vp, _vp, _vp, _vp],
        "hvx_min_max_loc": [_vp, _vp, _vp, _vp, _vp, ctypes.c_uint32, _vp],
        "hvx_buffer_from_ptr": [_vp, _vp, ctypes.c_size_t, _P(_vp)],
        "hvx_histogram_node": [_vp, _vp, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, _vp, _P(_vp)],
        "hvx_min_max_node": [_vp, _vp, _vp, _P(_vp)],
        "hvx_min_max_loc_node": [_vp, _vp, _vp, _vp, ctypes.c_uint32, _P(_vp)],
        "hvx_mean_std_dev_node": [_vp, _vp, _vp, _P(_vp)],
        "hvx_equalize_hist_node": [_vp, _vp, _vp, _P(_vp)],
        "hvx_box5x5_f32_node": [_vp, _vp, _vp, _P(_vp)],
        "hvx_sobel3x3_node": [_vp, _vp, _vp, _vp, _P(_vp)],
        "hvx_magnitude_node": [_vp, _vp, _vp, _vp, _P(_vp)],
        "hvx_phase_node": [_vp, _vp, _vp, _vp, _P(_vp)],
        "hvx_add_node": [_vp, _vp, _vp, ctypes.c_int, _vp, _P(_vp)],
        "hvx_multiply_f32_node": [_vp, _vp, _vp, _vp, _P(_vp)],
        "hvx_harris_response_node": [_vp, _vp, _vp, _vp, ctypes.c_float, _vp, _P(_vp)],
        "hvx_threshold_node": [_vp, _vp, ctypes.c_double, ctypes.c_uint8, ctypes.c_uint8, _vp, _P(_vp)],
        "hvx_convolve_node": [_vp, _vp, _vp, _vp, _P(_vp)],
        "hvx_node_set_border": [_vp, ctypes.c_int, ctypes.c_uint32],
        "hvx_graph_set_option": [_vp, ctypes.c_int, ctypes.c_int64],
        "hvx_graph_verify": [_vp],
        "hvx_graph_process": [_vp],
        "hvx_graph_schedule": [_vp, _vp],
        "hvx_graph_wait": [_vp],
        "hvx_graph_query": [_vp, ctypes.c_int, _P(ctypes.c_int64)],
        "hvx_graph_autotune": [_vp, _vp, ctypes.c_int],
        "hvx_context_save_tune_cache": [_vp, ctypes.c_char_p],
        "hvx_context_load_tune_cache": [_vp, ctypes.c_char_p],
        "hvx_batch_create": [_vp, _P(_vp), ctypes.c_uint32, _P(_vp)],
        "hvx_batch_refresh": [_vp],
        "hvx_batch_schedule": [_vp, _vp],
        "hvx_process_batch": [_vp, _P(_vp), ctypes.c_uint32, _vp],
        "hvx_batch_query": [_vp, ctypes.c_int, _P(ctypes.c_int64)],
        "hvx_batch_set_option": [_vp, ctypes.c_int, ctypes.c_int64],
        "hvx_batch_autotune": [_vp, _vp, ctypes.c_int],
        "hvx_server_create": [_vp, ctypes.c_int, ctypes.c_size_t, ctypes.c_uint32, ctypes.c_uint32, _P(_vp)],
        "hvx_server_submit": [_vp, _vp, _vp, ctypes.c_size_t, _vp, ctypes.c_size_t, ctypes.c_uint64],
        "hvx_server_submit_bound": [_vp, _vp, _P(hvx_binding), ctypes.c_uint32, ctypes.c_int, ctypes.c_uint64],
        "hvx_server_poll": [_vp, _P(ctypes.c_uint64), _P(ctypes.c_int32), _P(ctypes.c_double), ctypes.c_uint32,
                            _P(ctypes.c_uint32)],
        "hvx_server_drain": [_vp],
        "hvx_server_stats": [_vp, ctypes.c_int, _P(ctypes.c_int64)],
        "hvx_server_inject_failure": [_vp, ctypes.c_uint64],
        "hvx_release_graph": [_P(_vp)],
        "hvx_release_image": [_P(_vp)],
        "hvx_release_node": [_P(_vp)],
        "hvx_release_convolution": [_P(_vp)],
        "hvx_release_batch": [_P(_vp)],
        "hvx_release_server": [_P(_vp)],
        "hvx_release_buffer": [_P(_vp)],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int32
    lib.hvx_last_error.argtypes = [_vp]
    lib.hvx_last_error.restype = ctypes.c_char_p
    lib.hvx_status_name.argtypes = [ctypes.c_int32]
    lib.hvx_status_name.restype = ctypes.c_char_p
    _lib = lib
    return lib


def lib():
    return _load()


def status_name(s: int) -> str:
    return _load().hvx_status_name(s).decode()


def hvx_last_error(ctx) -> str:
    return _load().hvx_last_error(ctx).decode()


def _check(status, ctx=None):
    if status != 0:
        msg = hvx_last_error(ctx) if ctx else ""
        raise HvxError(status, msg)


def _out(fn, ctx, *args):
    h = _vp()
    _check(fn(*args, ctypes.byref(h)), ctx)
    return h.value


# ---- context, images -----------------------------------------------------------

def hvx_context_create(device: int = 0):
    return _out(_load().hvx_context_create, None, device)


def hvx_context_release(ctx):
    h = _vp(ctx)
    _check(_load().hvx_context_release(ctypes.byref(h)))


def hvx_image_from_ptr(ctx, w, h, df, ptr, pitch):
    return _out(_load().hvx_image_from_ptr, ctx, ctx, w, h, df, ptr, pitch)


def hvx_image_create(ctx, w, h, df):
    return _out(_load().hvx_image_create, ctx, ctx, w, h, df)


def hvx_image_swap_ptr(img, ptr, pitch, ctx=None):
    _check(_load().hvx_image_swap_ptr(img, ptr, pitch), ctx)


def hvx_image_query(img):
    w, h, df, p, pitch = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_int(), _vp(), ctypes.c_size_t()
    _check(_load().hvx_image_query(img, ctypes.byref(w), ctypes.byref(h), ctypes.byref(df), ctypes.byref(p),
                                   ctypes.byref(pitch)))
    return w.value, h.value, df.value, p.value, pitch.value


def hvx_image_copy(img, host_ptr, host_pitch, to_device, ctx=None):
    _check(_load().hvx_image_copy(img, host_ptr, host_pitch, int(to_device)), ctx)


def hvx_image_create_virtual(graph, w=0, h=0, df=HVX_DF_VIRT, ctx=None):
    return _out(_load().hvx_image_create_virtual, ctx, graph, w, h, df)


def hvx_convolution_create(ctx, coeffs, scale):
    import numpy as np
    c = np.ascontiguousarray(coeffs, dtype=np.int16)
    rows, cols = c.shape
    return _out(_load().hvx_convolution_create, ctx, ctx, cols, rows,
                c.ctypes.data_as(_P(ctypes.c_int16)), scale)


# ---- graph and nodes ---------------------------------------------------------------

def hvx_graph_create(ctx):
    return _out(_load().hvx_graph_create, ctx, ctx)


def _node(name, ctx, *args):
    return _out(getattr(_load(), name), ctx, *args)


def hvx_channel_extract_node(g, uyvy, channel, out, ctx=None):
    return _node("hvx_channel_extract_node", ctx, g, uyvy, channel, out)


def hvx_gaussian3x3_node(g, i, o, ctx=None):
    return _node("hvx_gaussian3x3_node", ctx, g, i, o)


def hvx_gaussian5x5_node(g, i, o, ctx=None):
    return _node("hvx_gaussian5x5_node", ctx, g, i, o)


def hvx_box3x3_node(g, i, o, ctx=None):
    return _node("hvx_box3x3_node", ctx, g, i, o)


def hvx_dilate3x3_node(g, i, o, ctx=None):
    return _node("hvx_dilate3x3_node", ctx, g, i, o)


def hvx_erode3x3_node(g, i, o, ctx=None):
    return _node("hvx_erode3x3_node", ctx, g, i, o)


def hvx_median3x3_node(g, i, o, ctx=None):
    return _node("hvx_median3x3_node", ctx, g, i, o)


HVX_NONLINEAR_MEDIAN, HVX_NONLINEAR_MIN, HVX_NONLINEAR_MAX = 0, 1, 2


def hvx_nonlinear_filter_node(g, function, i, mask, o, ctx=None):
    """`mask`: 2-D array (rows x cols, odd, at most 5x5); nonzero entries
    select window pixels."""
    import numpy as np
    m = np.ascontiguousarray((np.asarray(mask) != 0).astype(np.uint8))
    rows, cols = m.shape
    return _node("hvx_nonlinear_filter_node", ctx, g, function, i, cols, rows, m.ctypes.data_as(_vp), o)


def hvx_non_max_suppression_node(g, i, win_size, o, ctx=None):
    return _node("hvx_non_max_suppression_node", ctx, g, i, win_size, o)


def hvx_custom_point_node(g, expr, inputs, out_format, o, ctx=None):
    """User point kernel: `expr` over the images `inputs` (1 to 3, named a,
    b, c); `out_format` one of HVX_DF_U8 / S16 / F32."""
    arr = (_vp * len(inputs))(*inputs)
    return _node("hvx_custom_point_node", ctx, g, expr.encode(), arr, len(inputs), out_format, o)


def hvx_histogram(ctx, img, num_bins, offset, rng, dev_counts, stream=None):
    """Global operator: counts of a U8 image into `dev_counts` (device pointer
    to num_bins uint32), asynchronous on `stream`."""
    _check(_load().hvx_histogram(ctx, img, num_bins, offset, rng, dev_counts, stream), ctx)


def hvx_min_max(ctx, img, dev_min_max, stream=None):
    _check(_load().hvx_min_max(ctx, img, dev_min_max, stream), ctx)


def hvx_min_max_count(ctx, img, dev_result, stream=None):
    _check(_load().hvx_min_max_count(ctx, img, dev_result, stream), ctx)


def hvx_min_max_loc(ctx, img, dev_result, dev_min_locs, dev_max_locs, capacity, stream=None):
    _check(_load().hvx_min_max_loc(ctx, img, dev_result, dev_min_locs, dev_max_locs, capacity, stream), ctx)


def hvx_equalize_hist(ctx, img, out, dev_workspace, stream=None):
    _check(_load().hvx_equalize_hist(ctx, img, out, dev_workspace, stream), ctx)


def hvx_equalize_hist_noalloc(ctx, img, out, stream=None):
    _check(_load().hvx_equalize_hist_noalloc(ctx, img, out, stream), ctx)


def hvx_mean_std_dev(ctx, img, dev_result, stream=None):
    _check(_load().hvx_mean_std_dev(ctx, img, dev_result, stream), ctx)


def hvx_buffer_from_ptr(ctx, ptr, nbytes):
    """Wrap `nbytes` of caller-owned device memory (8-byte aligned) as the
    result buffer of a global operator node."""
    return _out(_load().hvx_buffer_from_ptr, ctx, ctx, ptr, nbytes)


def hvx_histogram_node(g, i, num_bins, offset, rng, counts, ctx=None):
    return _node("hvx_histogram_node", ctx, g, i, num_bins, offset, rng, counts)


def hvx_min_max_node(g, i, result, ctx=None):
    return _node("hvx_min_max_node", ctx, g, i, result)


def hvx_min_max_loc_node(g, i, result, locations, capacity, ctx=None):
    return _node("hvx_min_max_loc_node", ctx, g, i, result, locations, capacity)


def hvx_mean_std_dev_node(g, i, result, ctx=None):
    return _node("hvx_mean_std_dev_node", ctx, g, i, result)


def hvx_equalize_hist_node(g, i, o, ctx=None):
    return _node("hvx_equalize_hist_node", ctx, g, i, o)


def hvx_custom_local_node(g, expr, i, out_format, o, ctx=None):
    """User local kernel: `expr` over the window of image `i` (a[dx, dy])."""
    return _node("hvx_custom_local_node", ctx, g, expr.encode(), i, out_format, o)


def hvx_box5x5_f32_node(g, i, o, ctx=None):
    return _node("hvx_box5x5_f32_node", ctx, g, i, o)


def hvx_sobel3x3_node(g, i, gx, gy, ctx=None):
    return _node("hvx_sobel3x3_node", ctx, g, i, gx, gy)


def hvx_magnitude_node(g, gx, gy, o, ctx=None):
    return _node("hvx_magnitude_node", ctx, g, gx, gy, o)


def hvx_phase_node(g, gx, gy, o, ctx=None):
    return _node("hvx_phase_node", ctx, g, gx, gy, o)


def hvx_add_node(g, a, b, policy, o, ctx=None):
    return _node("hvx_add_node", ctx, g, a, b, policy, o)


def hvx_multiply_f32_node(g, a, b, o, ctx=None):
    return _node("hvx_multiply_f32_node", ctx, g, a, b, o)


def hvx_harris_response_node(g, sxx, syy, sxy, k, o, ctx=None):
    return _node("hvx_harris_response_node", ctx, g, sxx, syy, sxy, k, o)


def hvx_threshold_node(g, i, value, true_v, false_v, o, ctx=None):
    return _node("hvx_threshold_node", ctx, g, i, value, true_v, false_v, o)


def hvx_convolve_node(g, i, conv, o, ctx=None):
    return _node("hvx_convolve_node", ctx, g, i, conv, o)


def hvx_node_set_border(node, border, constant=0, ctx=None):
    _check(_load().hvx_node_set_border(node, border, constant), ctx)


def hvx_graph_set_option(g, option, value, ctx=None):
    _check(_load().hvx_graph_set_option(g, option, value), ctx)


def hvx_graph_verify(g, ctx=None):
    _check(_load().hvx_graph_verify(g), ctx)


def hvx_graph_process(g, ctx=None):
    _check(_load().hvx_graph_process(g), ctx)


def hvx_graph_schedule(g, stream=None, ctx=None):
    _check(_load().hvx_graph_schedule(g, stream), ctx)


def hvx_graph_wait(g, ctx=None):
    _check(_load().hvx_graph_wait(g), ctx)


def hvx_graph_query(g, attr, ctx=None) -> int:
    v = ctypes.c_int64()
    _check(_load().hvx_graph_query(g, attr, ctypes.byref(v)), ctx)
    return v.value


def hvx_graph_autotune(g, stream=None, iters=5, ctx=None):
    _check(_load().hvx_graph_autotune(g, stream, iters), ctx)


def hvx_context_save_tune_cache(ctx, path):
    _check(_load().hvx_context_save_tune_cache(ctx, path.encode()), ctx)


def hvx_context_load_tune_cache(ctx, path):
    _check(_load().hvx_context_load_tune_cache(ctx, path.encode()), ctx)


# ---- batches and serving -------------------------------------------------------------

def _handles(graphs):
    arr = (_vp * len(graphs))(*graphs)
    return arr


def hvx_batch_create(ctx, graphs):
    return _out(_load().hvx_batch_create, ctx, ctx, _handles(graphs), len(graphs))


def hvx_batch_refresh(b, ctx=None):
    _check(_load().hvx_batch_refresh(b), ctx)


def hvx_batch_schedule(b, stream=None, ctx=None):
    _check(_load().hvx_batch_schedule(b, stream), ctx)


def hvx_process_batch(ctx, graphs, stream=None):
    _check(_load().hvx_process_batch(ctx, _handles(graphs), len(graphs), stream), ctx)


def hvx_batch_query(b, attr, ctx=None) -> int:
    v = ctypes.c_int64()
    _check(_load().hvx_batch_query(b, attr, ctypes.byref(v)), ctx)
    return v.value


def hvx_batch_set_option(b, option, value, ctx=None):
    _check(_load().hvx_batch_set_option(b, option, value), ctx)


def hvx_batch_autotune(b, stream=None, iters=3, ctx=None):
    _check(_load().hvx_batch_autotune(b, stream, iters), ctx)


def hvx_server_create(ctx, mode, budget_bytes, max_slots, n_streams):
    return _out(_load().hvx_server_create, ctx, ctx, mode, budget_bytes, max_slots, n_streams)


def hvx_server_submit(s, templ, in_ptr, in_pitch, out_ptr, out_pitch, tag, ctx=None):
    _check(_load().hvx_server_submit(s, templ, in_ptr, in_pitch, out_ptr, out_pitch, tag), ctx)


def hvx_server_submit_bound(s, templ, bindings, memory, tag, ctx=None):
    """Queue a request; `bindings` lists (template image, pointer, pitch) for
    every non-virtual image of the template, in `memory` (HVX_MEMORY_HOST or
    HVX_MEMORY_DEVICE)."""
    arr = (hvx_binding * max(1, len(bindings)))(*[hvx_binding(i, p, pt) for (i, p, pt) in bindings])
    _check(_load().hvx_server_submit_bound(s, templ, arr, len(bindings), memory, tag), ctx)


def hvx_server_poll(s, max_n=256, ctx=None):
    tags = (ctypes.c_uint64 * max_n)()
    st = (ctypes.c_int32 * max_n)()
    lat = (ctypes.c_double * max_n)()
    n = ctypes.c_uint32()
    _check(_load().hvx_server_poll(s, tags, st, lat, max_n, ctypes.byref(n)), ctx)
    return [(tags[i], st[i], lat[i]) for i in range(n.value)]


def hvx_server_drain(s, ctx=None):
    _check(_load().hvx_server_drain(s), ctx)


def hvx_server_stats(s, what, ctx=None) -> int:
    v = ctypes.c_int64()
    _check(_load().hvx_server_stats(s, what, ctypes.byref(v)), ctx)
    return v.value


def hvx_server_inject_failure(s, tag, ctx=None):
    _check(_load().hvx_server_inject_failure(s, tag), ctx)


def _release(name, h):
    v = _vp(h)
    _check(getattr(_load(), name)(ctypes.byref(v)))


def hvx_release_graph(h):
    _release("hvx_release_graph", h)


def hvx_release_image(h):
    _release("hvx_release_image", h)


def hvx_release_node(h):
    _release("hvx_release_node", h)


def hvx_release_convolution(h):
    _release("hvx_release_convolution", h)


def hvx_release_batch(h):
    _release("hvx_release_batch", h)


def hvx_release_server(h):
    _release("hvx_release_server", h)


def hvx_release_buffer(h):
    _release("hvx_release_buffer", h)


# ---- torch marshalling helpers ----------------------------------------------------------

def alloc_image(h, w, df, device="cuda"):
    """A device image buffer with a 64-byte-aligned pitch: returns
    (buffer, view) where ``view`` is the (h, w) pixel view (UYVY: (h, 2w)
    bytes) and ``buffer`` the full (h, pitch) storage."""
    import torch
    dt = {HVX_DF_U8: torch.uint8, HVX_DF_S16: torch.int16, HVX_DF_S32: torch.int32, HVX_DF_F32: torch.float32,
          HVX_DF_UYVY: torch.uint8}[df]
    bpp = BYTES_PER_PIXEL[df]
    pitch = max(64, (w * bpp + 63) // 64 * 64)
    item = torch.empty((), dtype=dt).element_size()
    buf = torch.zeros((h, pitch // item), dtype=dt, device=device)
    cols = (w * bpp) // item
    return buf, buf[:, :cols]


def tensor_args(t):
    """(device pointer, pitch in bytes) of a 2-D tensor view."""
    return t.data_ptr(), t.stride(0) * t.element_size()


def image_from_tensor(ctx, t, df, w=None):
    """Wrap a 2-D device tensor (rows x pixels, UYVY as rows x 2*pixels bytes)."""
    ptr, pitch = tensor_args(t)
    h = t.shape[0]
    if w is None:
        w = t.shape[1] * t.element_size() // BYTES_PER_PIXEL[df]
    return hvx_image_from_ptr(ctx, w, h, df, ptr, pitch)
