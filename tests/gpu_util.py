"""Helpers for GPU tests: run a graph spec through libhvx on the device and
compare with the oracle.  Test infrastructure only."""
from __future__ import annotations

import sys

import numpy as np

import oracle
import paper_2008_11476_amd as hvx
import synth
from tests import graphspec as gs


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def device_image(ctx, arr, df, seed=0):
    """Upload `arr` into a pitched device buffer whose padding is random."""
    import torch
    host = synth.padded(arr, seed=seed)
    t = torch.from_numpy(np.ascontiguousarray(host)).cuda()
    h = arr.shape[0]
    w = arr.shape[1] // 2 if df == hvx.HVX_DF_UYVY else arr.shape[1]
    pitch = t.stride(0) * t.element_size()
    return hvx.hvx_image_from_ptr(ctx, w, h, df, t.data_ptr(), pitch), t


def run_spec(spec: gs.Spec, ctx, fusion=True, specialize=True, rows=0, dce=True, xcd=True, autotune=False,
             keep=None, codegen=True):
    """Execute `spec` on the GPU; returns ({output name: numpy array}, graph).
    `keep`, a dict, receives the device tensors (inputs, outputs, buffers) so
    that the graph can be processed again."""
    import torch
    imgs, keep_in, shapes = {}, [], {}
    for name, arr in spec.inputs.items():
        df = hvx.HVX_DF_UYVY if name in spec.uyvy else gs.DF_OF_DTYPE[arr.dtype]
        im, t = device_image(ctx, arr, df, seed=len(keep_in) + 1)
        imgs[name] = im
        keep_in.append(t)
        h = arr.shape[0]
        w = arr.shape[1] // 2 if df == hvx.HVX_DF_UYVY else arr.shape[1]
        shapes[name] = (h, w)
    h, w = next(iter(shapes.values()))
    outs = {}
    for i, (name, dt) in enumerate(spec.outputs.items()):
        dt = np.dtype(dt)
        garbage = np.random.default_rng(100 + i).integers(0, 255, size=(h, w)).astype(dt)
        df = gs.DF_OF_DTYPE[dt]
        im, t = device_image(ctx, garbage, df, seed=200 + i)
        imgs[name] = im
        outs[name] = (t, w, dt)
    bufs = {}
    for name, nbytes in spec.buffers.items():
        t = torch.full((nbytes,), 0x5A, dtype=torch.uint8, device="cuda")  # stale contents are overwritten
        imgs[name] = hvx.hvx_buffer_from_ptr(ctx, t.data_ptr(), nbytes)
        bufs[name] = t
    g, _, _ = gs.build_hvx(spec, ctx, imgs)
    hvx.hvx_graph_set_option(g, hvx.HVX_OPT_FUSION, int(fusion))
    hvx.hvx_graph_set_option(g, hvx.HVX_OPT_SPECIALIZE, int(specialize))
    hvx.hvx_graph_set_option(g, hvx.HVX_OPT_DCE, int(dce))
    hvx.hvx_graph_set_option(g, hvx.HVX_OPT_XCD_REMAP, int(xcd))
    hvx.hvx_graph_set_option(g, hvx.HVX_OPT_CODEGEN, int(codegen))
    if rows:
        hvx.hvx_graph_set_option(g, hvx.HVX_OPT_TILE, rows)
    hvx.hvx_graph_verify(g, ctx=ctx)
    if autotune:
        hvx.hvx_graph_autotune(g, torch.cuda.current_stream().cuda_stream, 2, ctx=ctx)
    hvx.hvx_graph_process(g, ctx=ctx)
    torch.cuda.synchronize()
    res = {}
    for name, (t, ww, dt) in outs.items():
        a = t.cpu().numpy()
        res[name] = a.view(dt)[:, :ww] if a.dtype != dt else a[:, :ww]
    for name, t in bufs.items():
        res[name] = t.cpu().numpy()  # raw bytes
    if keep is not None:
        keep.update({"inputs": keep_in, "outputs": outs, "buffers": bufs})
    return res, g


def circ_diff(a, b):
    d = np.abs(a.astype(np.int32) - b.astype(np.int32)) % 256
    return np.minimum(d, 256 - d)


def corner_ambiguous(env, thresh=1e6, k=0.04, rel=1e-5):
    """Pixels whose thresholded corner response may legitimately differ:
    |R - thresh| within the tolerance band rel * M (M bounds the terms)."""
    sxx, syy, sxy = env["sxx"], env["syy"], env["sxy"]
    m = np.abs(sxx * syy) + sxy * sxy + k * (sxx + syy) ** 2
    return np.abs(env["r"] - thresh) <= rel * m + 1e-3


def compare(spec: gs.Spec, got: dict, env: dict, exact_names=None, phase_names=(), corner=False):
    """Assert the GPU outputs equal the oracle's (phase within one level,
    corner threshold exact outside the tolerance band).  Only pixels that are
    specified (UNDEFINED borders) are compared."""
    valid = oracle.valid_masks(spec.oracle_graph(), spec.shapes())
    for name in spec.outputs:
        ref = env[name]
        out = got[name]
        assert out.shape == ref.shape, (name, out.shape, ref.shape)
        m = valid[name]
        if name in phase_names:
            d = circ_diff(out, ref)[m]
            assert d.size == 0 or d.max() <= 1, "%s: phase off by %d" % (name, d.max())
        elif corner:
            amb = corner_ambiguous(env)
            bad = (out != ref) & m & ~amb
            assert not bad.any(), "%s: %d corner pixels differ outside the tolerance band" % (name, bad.sum())
        else:
            bad = (out != ref) & m
            if bad.any():
                ys, xs = np.nonzero(bad)
                raise AssertionError("%s: %d pixels differ, first at (x=%d, y=%d): got %s want %s" % (
                    name, bad.sum(), xs[0], ys[0], out[ys[0], xs[0]], ref[ys[0], xs[0]]))
