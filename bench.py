"""Benchmark: the fused OpenVX-style Sobel-edge graph with its Phase branch on
4K frames, one MI355X.

One step = one execution of the verified graph Gaussian3x3 -> Sobel3x3 ->
{Magnitude -> Threshold at 100, Phase} (REPLICATE borders; two U8 outputs)
over F distinct 3840x2160 U8 frames resident in HBM (3 B/px, >= 1.5 GB of
distinct buffers, so the 256 MB last-level cache cannot serve them), issued
as one batch launch (a single kernel, so no HIP graph).  value = MPix/s of
the whole job.  The JSON line also reports the roofline of that kernel, the
CPU oracle on a bounded sample, and context measurements under "extras": the
same graph without Phase (2 B/px), 8K frames, CONSTANT(0) borders,
single-frame latency, node-by-node (unfused) execution, the corner graph at
1080p, the 256-image mixed batch and the serving loop against plain
per-request execution.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# VALU issue: 256 CUs x 4 SIMDs, one wave64 instruction per SIMD per 4 cycles
VALU_SIMDS = 256 * 4
CLOCK_HZ = 2.4e9


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("kernels.hip", "dev_fast.hpp", "dev_phase.hpp", "hvx_desc.h"):
        with open(os.path.join(ROOT, "paper_2008_11476_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def make_frames(hvx, torch, w, h, n, n_out=1, seed0=0):
    """n distinct device frames (pitched) derived from up to 4 seeded base
    frames (frame i = base[i % 4] XOR a per-frame byte), plus n_out output
    buffers per frame.  Kernels here are data-independent, so the content
    only needs to be distinct memory."""
    import synth
    nb = min(n, 4)
    bases = [torch.from_numpy(synth.edge_image(w, h, seed=seed0 + i)).cuda() for i in range(nb)]
    inp, out = [], []
    for i in range(n):
        buf, view = hvx.alloc_image(h, w, hvx.HVX_DF_U8)
        base, x = synth.frame_recipe(i, nb)
        view.copy_(bases[base] ^ x)
        inp.append((buf, view))
        out.append([hvx.alloc_image(h, w, hvx.HVX_DF_U8) for _ in range(n_out)])
    torch.cuda.synchronize()
    return inp, out


def edge_graph(hvx, ctx, inp_view, outs, phase=False, fusion=True, border=None, handles=None):
    g = hvx.hvx_graph_create(ctx)
    if handles:  # (input image, output image) handles made by the caller
        a, o = handles
    else:
        a = hvx.image_from_tensor(ctx, inp_view, hvx.HVX_DF_U8)
        o = hvx.image_from_tensor(ctx, outs[0][1], hvx.HVX_DF_U8)
    v = [hvx.hvx_image_create_virtual(g) for _ in range(4)]
    nodes = [hvx.hvx_gaussian3x3_node(g, a, v[0]), hvx.hvx_sobel3x3_node(g, v[0], v[1], v[2])]
    hvx.hvx_magnitude_node(g, v[1], v[2], v[3])
    hvx.hvx_threshold_node(g, v[3], 100.0, 255, 0, o)
    if phase:
        hvx.hvx_phase_node(g, v[1], v[2], hvx.image_from_tensor(ctx, outs[1][1], hvx.HVX_DF_U8))
    if border is not None:
        for n in nodes:
            hvx.hvx_node_set_border(n, border[0], border[1])
    hvx.hvx_graph_set_option(g, hvx.HVX_OPT_FUSION, int(fusion))
    hvx.hvx_graph_verify(g, ctx=ctx)
    return g


def corner_graph(hvx, ctx, inp_view, outs, handles=None):
    g = hvx.hvx_graph_create(ctx)
    if handles:
        a, o = handles
    else:
        a = hvx.image_from_tensor(ctx, inp_view, hvx.HVX_DF_U8)
        o = hvx.image_from_tensor(ctx, outs[0][1], hvx.HVX_DF_U8)
    v = [hvx.hvx_image_create_virtual(g) for _ in range(9)]
    hvx.hvx_sobel3x3_node(g, a, v[0], v[1])
    hvx.hvx_multiply_f32_node(g, v[0], v[0], v[2])
    hvx.hvx_multiply_f32_node(g, v[1], v[1], v[3])
    hvx.hvx_multiply_f32_node(g, v[0], v[1], v[4])
    hvx.hvx_box5x5_f32_node(g, v[2], v[5])
    hvx.hvx_box5x5_f32_node(g, v[3], v[6])
    hvx.hvx_box5x5_f32_node(g, v[4], v[7])
    hvx.hvx_harris_response_node(g, v[5], v[6], v[7], 0.04, v[8])
    hvx.hvx_threshold_node(g, v[8], 1e6, 255, 0, o)
    hvx.hvx_graph_verify(g, ctx=ctx)
    return g


def gauss5_graph(hvx, ctx, inp_view, outs, uyvy=False, w=None, handles=None):
    g = hvx.hvx_graph_create(ctx)
    if handles:
        a, o = handles
    else:
        o = hvx.image_from_tensor(ctx, outs[0][1], hvx.HVX_DF_U8)
        a = hvx.image_from_tensor(ctx, inp_view, hvx.HVX_DF_UYVY if uyvy else hvx.HVX_DF_U8, w=w)
    if uyvy:
        y = hvx.hvx_image_create_virtual(g)
        hvx.hvx_channel_extract_node(g, a, hvx.HVX_CHANNEL_Y, y)
        hvx.hvx_gaussian5x5_node(g, y, o)
    else:
        hvx.hvx_gaussian5x5_node(g, a, o)
    hvx.hvx_graph_verify(g, ctx=ctx)
    return g


def time_region(torch, fn, steps, warmup, spin_ms=150.0):
    """fn() repeated for `spin_ms` of wall time (the GPU leaves its idle
    clocks only under sustained load), then `warmup` more times, then `steps`
    timed calls: events on the current stream (the stream the kernels go to)
    and the host clock."""
    t_end = time.perf_counter() + spin_ms / 1e3
    while time.perf_counter() < t_end:
        for _ in range(8):
            fn()
        torch.cuda.synchronize()
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(s)
    for _ in range(steps):
        fn()
    e1.record(s)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    return e0.elapsed_time(e1) / steps, (t1 - t0) * 1e3 / steps


def batch_run(hvx, torch, ctx, graphs, steps, warmup, modes=("persistent", "direct"), rows=None):
    """Tune the batch's rows per work item (or pin them to `rows`), then time
    it in each launch mode; returns the fastest (ms, host ms, algorithmic
    bytes, mode, {mode: ms})."""
    stream = torch.cuda.current_stream().cuda_stream
    b = hvx.hvx_batch_create(ctx, graphs)
    if rows is None:
        hvx.hvx_batch_autotune(b, stream, 2, ctx=ctx)
    else:
        hvx.hvx_batch_set_option(b, hvx.HVX_BATCH_ROWS, rows, ctx=ctx)
    alg = hvx.hvx_batch_query(b, hvx.HVX_QUERY_ALG_BYTES)
    rows_item = hvx.hvx_batch_query(b, hvx.HVX_QUERY_ROWS_PER_ITEM)
    if rows_item == 0:
        # 0: each graph runs its own rows per item; report them when all agree
        own = {hvx.hvx_graph_query(g, hvx.HVX_QUERY_ROWS_PER_ITEM) for g in graphs}
        if len(own) == 1:
            rows_item = own.pop()
    per_mode = {"rows_per_item": rows_item, "work_items": hvx.hvx_batch_query(b, hvx.HVX_QUERY_NUM_OPS)}
    best = None
    for mode in modes:
        hvx.hvx_batch_set_option(b, hvx.HVX_BATCH_PERSISTENT, int(mode == "persistent"))
        ms, ms_host = time_region(torch, lambda: hvx.hvx_batch_schedule(b, stream, ctx=ctx), steps, warmup)
        per_mode[mode] = round(ms, 4)
        if best is None or ms < best[0]:
            best = (ms, ms_host, mode)
    hvx.hvx_release_batch(b)
    return best[0], best[1], alg, best[2], per_mode


def edge_batch(hvx, torch, ctx, w, h, nframes, steps, warmup, phase=False, border=None, rows=None,
               modes=("persistent", "direct")):
    inp, out = make_frames(hvx, torch, w, h, nframes, n_out=2 if phase else 1)
    graphs = [edge_graph(hvx, ctx, inp[i][1], out[i], phase=phase, border=border) for i in range(nframes)]
    ms, ms_host, alg, mode, per_mode = batch_run(hvx, torch, ctx, graphs, steps, warmup, modes=modes, rows=rows)
    for g in graphs:
        hvx.hvx_release_graph(g)
    del inp, out
    torch.cuda.empty_cache()
    mpix = nframes * w * h / 1e6
    return dict(ms=ms, ms_host=ms_host, alg_bytes=alg, mpix_s=mpix / (ms / 1e3), gbs=alg / (ms / 1e3) / 1e9,
                rows=per_mode["rows_per_item"], mode=mode, per_mode=per_mode)


def kind_counters(name, kernel, rows, ms):
    """frac and VALU issue fraction of one profiled batch launch, from the
    committed counter summary profiles/<name>_counters.json (written from
    rocprofv3 runs of `bench.py --only <name>`), used only while its hash
    matches the kernel sources and it holds the launch's rows per item."""
    f = os.path.join(ROOT, "profiles", name + "_counters.json")
    if not os.path.exists(f):
        return {}
    c = json.load(open(f))
    if c.get("kernel_hash") != kernel_source_hash() or c.get("kernel") != kernel:
        return {}
    e = c.get("shapes", {}).get(str(rows))
    if not e:
        return {}
    out = {}
    if e.get("valu_insts_per_launch"):
        out["valu_issue_frac"] = round(e["valu_insts_per_launch"] / (VALU_SIMDS * (ms * 1e-3) * CLOCK_HZ / 4), 4)
    if e.get("bytes_per_launch"):
        out["traffic_bytes"] = e["bytes_per_launch"]
    return out


def batch_kernel(per_mode, kinds):
    """Name of the batch kernel a measurement ran (direct or persistent)."""
    direct = per_mode.get("direct", 1e9) <= per_mode.get("persistent", 1e9)
    return "hvx::k_batch%s<%d>" % ("_direct" if direct else "", kinds)


def ex_edge_4k_batch64(hvx, torch, ctx, rec, rows=None):
    # the graph without its Phase branch (2 B/px), 64 4K frames
    r = edge_batch(hvx, torch, ctx, 3840, 2160, 64, 20, 3, rows=rows, modes=("direct",) if rows else
                   ("persistent", "direct"))
    d = {"mpix_s": round(r["mpix_s"], 1), "alg_gbs": round(r["gbs"], 1), "hbm_frac": round(r["gbs"] / HBM_PEAK_GBS, 4),
         "ms": round(r["ms"], 4), "rows": r["rows"], "batch_mode_ms": r["per_mode"]}
    d.update(kind_counters("edge_4k_batch64", batch_kernel(r["per_mode"], 1), r["rows"], r["ms"]))
    rec("edge_4k_batch64", d)


def ex_edge_phase_4k_latency(hvx, torch, ctx, rec):
    stream = torch.cuda.current_stream().cuda_stream
    # single 4K frame, one launch per frame (latency view)
    inp, out = make_frames(hvx, torch, 3840, 2160, 1, n_out=2)
    g = edge_graph(hvx, ctx, inp[0][1], out[0], phase=True)
    hvx.hvx_graph_autotune(g, stream, 5, ctx=ctx)
    ms, _ = time_region(torch, lambda: hvx.hvx_graph_schedule(g, stream, ctx=ctx), 50, 5)
    rec("edge_phase_4k_single_frame", {"us_per_frame": round(ms * 1e3, 2), "mpix_s": round(8.2944 / (ms / 1e3), 1),
                                       "rows_per_item": hvx.hvx_graph_query(g, hvx.HVX_QUERY_ROWS_PER_ITEM)})
    # node by node (fusion off): six kernels, intermediates in HBM
    gu = edge_graph(hvx, ctx, inp[0][1], out[0], phase=True, fusion=False)
    ms_u, _ = time_region(torch, lambda: hvx.hvx_graph_schedule(gu, stream, ctx=ctx), 20, 3)
    hbm_u = hvx.hvx_graph_query(gu, hvx.HVX_QUERY_HBM_BYTES)
    rec("edge_phase_4k_unfused", {"us_per_frame": round(ms_u * 1e3, 2), "mpix_s": round(8.2944 / (ms_u / 1e3), 1),
                                  "kernels": hvx.hvx_graph_query(gu, hvx.HVX_QUERY_NUM_KERNELS),
                                  "hbm_bytes_per_frame": hbm_u, "gbs": round(hbm_u / (ms_u / 1e3) / 1e9, 1),
                                  "fused_speedup_single_frame": round(ms_u / ms, 2)})
    for x in (g, gu):
        hvx.hvx_release_graph(x)
    del inp, out


def ex_edge_8k(hvx, torch, ctx, rec):
    r = edge_batch(hvx, torch, ctx, 7680, 4320, 16, 10, 2, phase=True)
    rec("edge_phase_8k_batch16", {"mpix_s": round(r["mpix_s"], 1), "alg_gbs": round(r["gbs"], 1),
                                  "ms": round(r["ms"], 3), "rows": r["rows"], "batch_mode_ms": r["per_mode"]})
    r = edge_batch(hvx, torch, ctx, 7680, 4320, 16, 10, 2)
    rec("edge_8k_batch16", {"mpix_s": round(r["mpix_s"], 1), "alg_gbs": round(r["gbs"], 1),
                            "ms": round(r["ms"], 3), "rows": r["rows"], "batch_mode_ms": r["per_mode"]})


def ex_edge_constant(hvx, torch, ctx, rec):
    r = edge_batch(hvx, torch, ctx, 3840, 2160, 64, 10, 2, phase=True, border=(hvx.HVX_BORDER_CONSTANT, 0))
    rec("edge_phase_4k_constant0_batch64", {"mpix_s": round(r["mpix_s"], 1), "alg_gbs": round(r["gbs"], 1),
                                            "ms": round(r["ms"], 3)})


def ex_gauss5(hvx, torch, ctx, rec, uyvy=False, rows=None):
    """Gaussian5x5 on 64 4K frames: U8 input (2 B/px) or UYVY input (3 B/px)."""
    import synth
    W4, H4, n = 3840, 2160, 64
    ins, outs = [], []
    for i in range(n):
        if uyvy:
            ib, iv = hvx.alloc_image(H4, W4, hvx.HVX_DF_UYVY)
            if i < 4:
                iv.copy_(torch.from_numpy(synth.uyvy_image(W4, H4, seed=i)))
            else:
                iv.copy_(ins[i % 4][1] ^ ((i // 4) * 37 % 256))
        else:
            ib, iv = hvx.alloc_image(H4, W4, hvx.HVX_DF_U8)
            if i < 4:
                iv.copy_(torch.from_numpy(synth.edge_image(W4, H4, seed=i)))
            else:
                iv.copy_(ins[i % 4][1] ^ ((i // 4) * 37 % 256))
        ins.append((ib, iv))
        outs.append([hvx.alloc_image(H4, W4, hvx.HVX_DF_U8)])
    graphs = [gauss5_graph(hvx, ctx, ins[i][1], outs[i], uyvy=uyvy, w=W4) for i in range(n)]
    ms, _, alg, mode, per_mode = batch_run(hvx, torch, ctx, graphs, 10, 2, rows=rows,
                                           modes=("direct",) if rows else ("persistent", "direct"))
    name = "uyvy_gauss5_4k_batch64" if uyvy else "gauss5_4k_batch64"
    d = {"mpix_s": round(n * W4 * H4 / 1e6 / (ms / 1e3), 1), "alg_gbs": round(alg / (ms / 1e3) / 1e9, 1),
         "hbm_frac": round(alg / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4), "ms": round(ms, 4), "batch_mode_ms": per_mode}
    d.update(kind_counters(name, batch_kernel(per_mode, 16 if uyvy else 4), per_mode["rows_per_item"], ms))
    rec(name, d)
    for x in graphs:
        hvx.hvx_release_graph(x)
    del ins, outs
    torch.cuda.empty_cache()


def ex_corner(hvx, torch, ctx, rec, rows=None):
    """Corner graph at 1080p: single frame and a 32-frame batch (2 B/px)."""
    stream = torch.cuda.current_stream().cuda_stream
    inp, out = make_frames(hvx, torch, 1920, 1080, 32)
    graphs = [corner_graph(hvx, ctx, inp[i][1], out[i]) for i in range(32)]
    hvx.hvx_graph_autotune(graphs[0], stream, 5, ctx=ctx)
    for x in graphs:
        hvx.hvx_graph_verify(x, ctx=ctx)
    ms1, _ = time_region(torch, lambda: hvx.hvx_graph_schedule(graphs[0], stream, ctx=ctx), 50, 5)
    ms, _, alg, mode, per_mode = batch_run(hvx, torch, ctx, graphs, 10, 2, rows=rows,
                                           modes=("direct",) if rows else ("persistent", "direct"))
    mp = 32 * 1920 * 1080 / 1e6
    d = {"us_single_frame": round(ms1 * 1e3, 2), "batch32_mpix_s": round(mp / (ms / 1e3), 1),
         "batch32_alg_gbs": round(alg / (ms / 1e3) / 1e9, 1),
         "hbm_frac": round(alg / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4), "batch32_ms": round(ms, 4),
         "batch_mode_ms": per_mode, "kernel_kind": hvx.hvx_graph_query(graphs[0], hvx.HVX_QUERY_KERNEL_KIND)}
    d.update(kind_counters("corner_1080p", batch_kernel(per_mode, 2), per_mode["rows_per_item"], ms))
    rec("corner_1080p", d)
    for x in graphs:
        hvx.hvx_release_graph(x)
    del inp, out
    torch.cuda.empty_cache()


def ex_mixed(hvx, torch, ctx, rec, rows=None):
    """256 images of random sizes and kinds in one launch."""
    import synth
    shapes = synth.batch_shapes(256, seed=0)
    keep, graphs = [], []
    total_px = 0
    for (w, h, kind, seed) in shapes:
        ib, iv = hvx.alloc_image(h, w, hvx.HVX_DF_U8)
        iv.copy_(torch.from_numpy(synth.uniform_u8(w, h, seed)))
        ob = hvx.alloc_image(h, w, hvx.HVX_DF_U8)
        keep += [ib, ob[0]]
        if kind == "sobel_edge":
            graphs.append(edge_graph(hvx, ctx, iv, [ob]))
        elif kind == "harris":
            graphs.append(corner_graph(hvx, ctx, iv, [ob]))
        else:
            graphs.append(gauss5_graph(hvx, ctx, iv, [ob]))
        total_px += w * h
    torch.cuda.synchronize()
    ms, ms_host, alg, mode, per_mode = batch_run(hvx, torch, ctx, graphs, 10, 2, rows=rows,
                                                 modes=("direct",) if rows else ("persistent", "direct"))
    d = {"mpix": round(total_px / 1e6, 1), "ms": round(ms, 3), "batch_mode_ms": per_mode,
         "mpix_s": round(total_px / 1e6 / (ms / 1e3), 1), "alg_gbs": round(alg / (ms / 1e3) / 1e9, 1),
         "hbm_frac": round(alg / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}
    d.update(kind_counters("mixed_batch256", batch_kernel(per_mode, 7), per_mode["rows_per_item"], ms))
    rec("mixed_batch256", d)
    for x in graphs:
        hvx.hvx_release_graph(x)
    del keep
    torch.cuda.empty_cache()


def res_set(rec, name, d):
    rec(name, d)


# named context measurements (`--only NAME` runs one of them without the headline)
EXTRAS = {
    "edge_4k_batch64": ex_edge_4k_batch64,
    "edge_phase_4k_latency": ex_edge_phase_4k_latency,
    "edge_8k": ex_edge_8k,
    "edge_constant": ex_edge_constant,
    "gauss5_4k_batch64": lambda hvx, torch, ctx, rec, rows=None: ex_gauss5(hvx, torch, ctx, rec, rows=rows),
    "uyvy_gauss5_4k_batch64": lambda hvx, torch, ctx, rec, rows=None: ex_gauss5(hvx, torch, ctx, rec, uyvy=True,
                                                                                 rows=rows),
    "corner_1080p": ex_corner,
    "mixed_batch256": ex_mixed,
    "global_ops_16k": lambda hvx, torch, ctx, rec: global_ops(hvx, torch, ctx, torch.cuda.current_stream().cuda_stream,
                                                              rec),
    "global_graph_4k": lambda hvx, torch, ctx, rec: global_graph(hvx, torch, ctx, rec),
    "user_kernels_4k": lambda hvx, torch, ctx, rec: user_kernels(hvx, torch, ctx, rec),
    # the generated kernels alone (one fused plan per graph, default tiles): the profiled command
    "user_kernels_fused_4k": lambda hvx, torch, ctx, rec: user_kernels(hvx, torch, ctx, rec, fused_only=True),
    "user_kernels_4k_batch32": lambda hvx, torch, ctx, rec: user_kernels_batch(hvx, torch, ctx, rec),
    "serving": lambda hvx, torch, ctx, rec: res_set(rec, "serving", serving(hvx, torch, ctx)),
}


def extras(hvx, torch, ctx, only=None, rows=None):
    res = {}

    def rec(name, d):
        res[name] = d
        log(name, json.dumps(d))

    for name, fn in EXTRAS.items():
        if only and name not in only:
            continue
        if rows is not None:
            fn(hvx, torch, ctx, rec, rows=rows)
        else:
            fn(hvx, torch, ctx, rec)
    return res


def global_ops(hvx, torch, ctx, stream, rec):
    """Global operators (Table 2) over one 16384 x 16384 U8 image: one read
    pass of 268 MB each (EqualizeHist also writes 268 MB; MinMaxLoc keeps at
    most 1024 locations of each extreme).  The timed call includes the kernel that initialises
    the result (and, for mean/stddev, the final kernel)."""
    gw = gh = 16384
    gb, gv = hvx.alloc_image(gh, gw, hvx.HVX_DF_U8)
    gv.copy_(torch.randint(0, 256, (gh, gw), dtype=torch.uint8, device="cuda"))
    gim = hvx.image_from_tensor(ctx, gv, hvx.HVX_DF_U8)
    gout = torch.zeros(1024, dtype=torch.int64, device="cuda")  # results (MinMaxLoc: 4128 bytes), then a workspace
    gloc = torch.zeros(4096, dtype=torch.int32, device="cuda")  # two lists of 1024 (x, y) pairs
    gob, gov = hvx.alloc_image(gh, gw, hvx.HVX_DF_U8)
    gom = hvx.image_from_tensor(ctx, gov, hvx.HVX_DF_U8)
    gops = {"histogram256": lambda: hvx.hvx_histogram(ctx, gim, 256, 0, 256, gout.data_ptr(), stream),
            "min_max": lambda: hvx.hvx_min_max(ctx, gim, gout.data_ptr(), stream),
            "min_max_count": lambda: hvx.hvx_min_max_count(ctx, gim, gout.data_ptr(), stream),
            "min_max_loc_cap1024": lambda: hvx.hvx_min_max_loc(ctx, gim, gout.data_ptr(), gloc.data_ptr(),
                                                               gloc.data_ptr() + 8192, 1024, stream),
            "equalize_hist": lambda: hvx.hvx_equalize_hist(ctx, gim, gom, gout.data_ptr() + 4160, stream),
            "mean_std_dev": lambda: hvx.hvx_mean_std_dev(ctx, gim, gout.data_ptr(), stream)}
    gd = {"image": "16384x16384 U8, uniform random", "alg_bytes": gw * gh}
    for name, fn in gops.items():
        ms, _ = time_region(torch, fn, 20, 3)
        gbs = gw * gh * (2 if name == "equalize_hist" else 1) / (ms / 1e3) / 1e9  # equalize also writes
        gd[name] = {"ms": round(ms, 4), "alg_gbs": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)}
    rec("global_ops_16k", gd)
    hvx.hvx_release_image(gim)
    hvx.hvx_release_image(gom)
    del gb, gv, gout, gloc, gob, gov
    torch.cuda.empty_cache()


def tuned_plan(hvx, torch, ctx, build, stream, pixels, alg_bytes):
    """The plan the autotuner picks for a graph (fused, cut at a value, or
    cut at every value; the generated kernels' tiles), timed like the fixed
    plans."""
    g = hvx.hvx_graph_create(ctx)
    build(g)
    hvx.hvx_graph_verify(g, ctx=ctx)
    hvx.hvx_graph_autotune(g, stream, 5, ctx=ctx)
    ms, _ = time_region(torch, lambda: hvx.hvx_graph_schedule(g, stream, ctx=ctx), 20, 3)
    tile = hvx.hvx_graph_query(g, hvx.HVX_QUERY_GEN_TILE)
    r = {"us": round(ms * 1e3, 2), "mpix_s": round(pixels / 1e6 / (ms / 1e3), 1),
         "kernels": hvx.hvx_graph_query(g, hvx.HVX_QUERY_NUM_KERNELS),
         "generated": hvx.hvx_graph_query(g, hvx.HVX_QUERY_NUM_GENERATED),
         "cut_values": hvx.hvx_graph_query(g, hvx.HVX_QUERY_PLAN_CUTS),
         "tile": "%dx%d" % (tile >> 16, tile & 0xFFFF) if tile else None,
         "alg_gbs": round(alg_bytes / (ms / 1e3) / 1e9, 1)}
    hvx.hvx_release_graph(g)
    return r


# plans compared by the graph measurements: (label, HVX_OPT_FUSION, HVX_OPT_CODEGEN)
PLANS = (("fused", 1, 1), ("fused_interpreted", 1, 0), ("node_by_node", 0, 1))


def global_graph(hvx, torch, ctx, rec):
    """Global operators as graph nodes on one 3840x2160 frame: Gaussian3x3 ->
    Histogram and Gaussian5x5 -> MinMaxLoc counts, the producer fused into the
    reduction (one generated kernel, 1 B/px read; and the same group run by
    the tile interpreter) against the same graphs node by node (the Gaussian
    written to memory and read back: 3 B/px)."""
    import synth
    stream = torch.cuda.current_stream().cuda_stream
    w, h = 3840, 2160
    ib, iv = hvx.alloc_image(h, w, hvx.HVX_DF_U8)
    iv.copy_(torch.from_numpy(synth.edge_image(w, h, seed=0)))
    img = hvx.image_from_tensor(ctx, iv, hvx.HVX_DF_U8)
    buf = torch.zeros(8192, dtype=torch.uint8, device="cuda")
    res = hvx.hvx_buffer_from_ptr(ctx, buf.data_ptr(), 8192)
    d = {"image": "3840x2160 U8"}
    for name, make in (("gauss3_histogram", lambda g, v: hvx.hvx_histogram_node(g, v, 256, 0, 256, res)),
                       ("gauss5_min_max_loc_counts", lambda g, v: hvx.hvx_min_max_loc_node(g, v, res, None, 0))):
        row = {}
        for label, fusion, codegen in PLANS:
            g = hvx.hvx_graph_create(ctx)
            v = hvx.hvx_image_create_virtual(g)
            if name.startswith("gauss3"):
                hvx.hvx_gaussian3x3_node(g, img, v)
            else:
                hvx.hvx_gaussian5x5_node(g, img, v)
            make(g, v)
            hvx.hvx_graph_set_option(g, hvx.HVX_OPT_FUSION, fusion)
            hvx.hvx_graph_set_option(g, hvx.HVX_OPT_CODEGEN, codegen)
            hvx.hvx_graph_verify(g, ctx=ctx)
            ms, _ = time_region(torch, lambda: hvx.hvx_graph_schedule(g, stream, ctx=ctx), 20, 3)
            hbm = hvx.hvx_graph_query(g, hvx.HVX_QUERY_HBM_BYTES)
            row[label] = {
                "us": round(ms * 1e3, 2), "mpix_s": round(w * h / 1e6 / (ms / 1e3), 1),
                "kernels": hvx.hvx_graph_query(g, hvx.HVX_QUERY_NUM_KERNELS),
                "generated": hvx.hvx_graph_query(g, hvx.HVX_QUERY_NUM_GENERATED), "hbm_bytes": hbm,
                "gbs": round(hbm / (ms / 1e3) / 1e9, 1)}
            hvx.hvx_release_graph(g)
        row["fused_speedup"] = round(row["node_by_node"]["us"] / row["fused"]["us"], 2)

        def build(g, name=name, make=make):
            v = hvx.hvx_image_create_virtual(g)
            if name.startswith("gauss3"):
                hvx.hvx_gaussian3x3_node(g, img, v)
            else:
                hvx.hvx_gaussian5x5_node(g, img, v)
            make(g, v)
        row["tuned"] = tuned_plan(hvx, torch, ctx, build, stream, w * h, w * h)
        d[name] = row
    rec("global_graph_4k", d)
    hvx.hvx_release_image(img)
    hvx.hvx_release_buffer(res)
    del ib, iv, buf


def user_kernel_builders(hvx, ctx):
    """Builders of the paper's user-kernel applications (Section 6.1), each
    adding its nodes to a graph between an input image a and an output image
    o (U8): Unsharp (Gaussian3x3 and three user point kernels), Tomasi (the
    corner graph with a user min-eigenvalue response), FChain (three Convolve
    nodes).  Returns the builders and the convolutions to release."""
    S16, F32, U8 = hvx.HVX_DF_S16, hvx.HVX_DF_F32, hvx.HVX_DF_U8

    def unsharp(g, a, o):
        v = [hvx.hvx_image_create_virtual(g) for _ in range(3)]
        hvx.hvx_gaussian3x3_node(g, a, v[0])
        hvx.hvx_custom_point_node(g, "a - b", [a, v[0]], S16, v[1])
        hvx.hvx_custom_point_node(g, "a * 3 / 2", [v[1]], S16, v[2])
        hvx.hvx_custom_point_node(g, "a + b", [a, v[2]], U8, o)

    def tomasi(g, a, o):
        v = [hvx.hvx_image_create_virtual(g) for _ in range(9)]
        hvx.hvx_sobel3x3_node(g, a, v[0], v[1])
        hvx.hvx_multiply_f32_node(g, v[0], v[0], v[2])
        hvx.hvx_multiply_f32_node(g, v[1], v[1], v[3])
        hvx.hvx_multiply_f32_node(g, v[0], v[1], v[4])
        for k in range(3):
            hvx.hvx_box5x5_f32_node(g, v[2 + k], v[5 + k])
        hvx.hvx_custom_point_node(g, "(a + b) / 2 - sqrt((a - b) * (a - b) / 4 + c * c)", [v[5], v[6], v[7]], F32,
                                  v[8])
        hvx.hvx_threshold_node(g, v[8], 2e5, 255, 0, o)

    masks = [(np.outer([1, 4, 6, 4, 1], [1, 4, 6, 4, 1]), 256), (np.array([[0, -1, 0], [-1, 5, -1], [0, -1, 0]]), 1),
             (np.ones((5, 5), int), 32)]
    convs = [hvx.hvx_convolution_create(ctx, m, sc) for (m, sc) in masks]

    def fchain(g, a, o):
        v = [hvx.hvx_image_create_virtual(g, 0, 0, U8) for _ in range(2)]
        hvx.hvx_convolve_node(g, a, convs[0], v[0])
        hvx.hvx_convolve_node(g, v[0], convs[1], v[1])
        hvx.hvx_convolve_node(g, v[1], convs[2], o)

    return (("unsharp", unsharp), ("tomasi", tomasi), ("fchain", fchain)), convs


def user_kernels(hvx, torch, ctx, rec, fused_only=False):
    """The user-kernel applications on one 3840x2160 frame, U8 in and U8 out
    (2 B/px), fused (one generated kernel; and the same group run by the tile
    interpreter) and node by node (user kernels generated one by one), and the
    plan the tuner picks."""
    import synth
    stream = torch.cuda.current_stream().cuda_stream
    w, h = 3840, 2160
    ib, iv = hvx.alloc_image(h, w, hvx.HVX_DF_U8)
    ob, ov = hvx.alloc_image(h, w, hvx.HVX_DF_U8)
    iv.copy_(torch.from_numpy(synth.corner_image(w, h, seed=0)))
    a = hvx.image_from_tensor(ctx, iv, hvx.HVX_DF_U8)
    o = hvx.image_from_tensor(ctx, ov, hvx.HVX_DF_U8)
    builders, convs = user_kernel_builders(hvx, ctx)
    d = {"image": "3840x2160 U8 (corner workload)", "alg_bytes_per_frame": 2 * w * h}
    for name, make in builders:
        def build(g, make=make):
            make(g, a, o)
        row = {}
        for label, fusion, codegen in PLANS[:1] if fused_only else PLANS:
            g = hvx.hvx_graph_create(ctx)
            build(g)
            hvx.hvx_graph_set_option(g, hvx.HVX_OPT_FUSION, fusion)
            hvx.hvx_graph_set_option(g, hvx.HVX_OPT_CODEGEN, codegen)
            hvx.hvx_graph_verify(g, ctx=ctx)
            ms, _ = time_region(torch, lambda: hvx.hvx_graph_schedule(g, stream, ctx=ctx), 20, 3)
            row[label] = {
                "us": round(ms * 1e3, 2), "mpix_s": round(w * h / 1e6 / (ms / 1e3), 1),
                "kernels": hvx.hvx_graph_query(g, hvx.HVX_QUERY_NUM_KERNELS),
                "generated": hvx.hvx_graph_query(g, hvx.HVX_QUERY_NUM_GENERATED),
                "alg_gbs": round(2 * w * h / (ms / 1e3) / 1e9, 1),
                "hbm_frac": round(2 * w * h / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
                "plan_hbm_bytes": hvx.hvx_graph_query(g, hvx.HVX_QUERY_HBM_BYTES)}
            hvx.hvx_release_graph(g)
        if not fused_only:
            row["fused_speedup"] = round(row["node_by_node"]["us"] / row["fused"]["us"], 2)
            row["tuned"] = tuned_plan(hvx, torch, ctx, build, stream, w * h, 2 * w * h)
        d[name] = row
    rec("user_kernels_fused_4k" if fused_only else "user_kernels_4k", d)
    for c in convs:
        hvx.hvx_release_convolution(c)
    hvx.hvx_release_image(a)
    hvx.hvx_release_image(o)
    del ib, iv, ob, ov


def user_kernels_batch(hvx, torch, _shared_ctx, rec, nframes=32):
    """The user-kernel applications over 32 distinct 3840x2160 frames in one
    batch: the graphs share their generated kernel, so each application is
    one launch over every frame's tiles (throughput rather than one frame's
    latency).  The graphs live in a context of their own, so they run the
    default plan rather than the plan tuned for one frame (a smaller tile
    that lowers one frame's latency and costs throughput over many)."""
    stream = torch.cuda.current_stream().cuda_stream
    w, h = 3840, 2160
    ctx = hvx.hvx_context_create(0)
    inp, out = make_frames(hvx, torch, w, h, nframes)
    builders, convs = user_kernel_builders(hvx, ctx)
    handles = [(hvx.image_from_tensor(ctx, inp[i][1], hvx.HVX_DF_U8),
                hvx.image_from_tensor(ctx, out[i][0][1], hvx.HVX_DF_U8)) for i in range(nframes)]
    d = {"frames": "%d x 3840x2160 U8" % nframes, "alg_bytes_per_step": 2 * w * h * nframes}
    for name, make in builders:
        graphs = []
        for a, o in handles:
            g = hvx.hvx_graph_create(ctx)
            make(g, a, o)
            hvx.hvx_graph_verify(g, ctx=ctx)
            graphs.append(g)
        b = hvx.hvx_batch_create(ctx, graphs)
        ms, _ = time_region(torch, lambda: hvx.hvx_batch_schedule(b, stream, ctx=ctx), 10, 2)
        alg = 2 * w * h * nframes
        d[name] = {"ms": round(ms, 4), "mpix_s": round(nframes * w * h / 1e6 / (ms / 1e3), 1),
                   "launches": hvx.hvx_batch_query(b, hvx.HVX_QUERY_NUM_KERNELS),
                   "alg_gbs": round(alg / (ms / 1e3) / 1e9, 1), "hbm_frac": round(alg / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}
        hvx.hvx_release_batch(b)
        for g in graphs:
            hvx.hvx_release_graph(g)
    rec("user_kernels_4k_batch32", d)
    for c in convs:
        hvx.hvx_release_convolution(c)
    for a, o in handles:
        hvx.hvx_release_image(a)
        hvx.hvx_release_image(o)
    hvx.hvx_context_release(ctx)
    del inp, out
    torch.cuda.empty_cache()


def serving(hvx, torch, ctx, n_req=240, budget=512 << 20):
    """Poisson request stream over {edge, corner, UYVY->Y+Gaussian5x5} x
    {640x480, 1280x720, 1920x1080, 3840x2160}, served two ways: frames
    resident in HBM (requests bound to device buffers and run in place) and
    host frames in pinned memory (copied in and out by the server).  For
    each: the plain loop's and the continuous loop's burst capacity, then
    arrival rates set from the plain capacity (0.5, 0.8, 0.95 and 1.2 of it),
    served continuously and plainly."""
    import synth
    templ, host_in, dev_in, dev_out, timg = {}, {}, {}, {}, {}
    keep = []
    for kind in synth.SERVE_TYPES:
        for (w, h) in synth.SERVE_SIZES:
            df = hvx.HVX_DF_UYVY if kind == "uyvy_gauss5" else hvx.HVX_DF_U8
            ib, iv = hvx.alloc_image(h, w, df)
            ob, ov = hvx.alloc_image(h, w, hvx.HVX_DF_U8)
            ih = hvx.image_from_tensor(ctx, iv, df, w=w)
            oh = hvx.image_from_tensor(ctx, ov, hvx.HVX_DF_U8)
            if kind == "uyvy_gauss5":
                g = gauss5_graph(hvx, ctx, None, None, uyvy=True, w=w, handles=(ih, oh))
                frame = synth.uyvy_image(w, h, seed=w)
            else:
                g = (edge_graph if kind == "sobel_edge" else corner_graph)(hvx, ctx, None, None, handles=(ih, oh))
                frame = synth.edge_image(w, h, seed=w)
            keep += [ib, ob]
            key = (kind, w, h)
            templ[key] = g
            timg[key] = (ih, oh)
            host_in[key] = torch.from_numpy(frame).pin_memory()
            # resident frames: 4 inputs and 8 outputs per template in HBM
            dev_in[key] = []
            for j in range(4):
                db, dv = hvx.alloc_image(h, w, df)
                dv.copy_(torch.from_numpy(frame) ^ j)
                keep.append(db)
                dev_in[key].append(dv)
            dev_out[key] = []
            for j in range(8):
                db, dv = hvx.alloc_image(h, w, hvx.HVX_DF_U8)
                keep.append(db)
                dev_out[key].append(dv)
    outs = {}
    for key in templ:
        outs[key] = [torch.empty((key[2], key[1]), dtype=torch.uint8).pin_memory() for _ in range(8)]
    torch.cuda.synchronize()

    def run(mode, trace, device, n_streams=2):
        s = hvx.hvx_server_create(ctx, mode, budget, 16, n_streams)
        t0 = time.perf_counter()
        lat = []
        px = 0
        for i, (ta, kind, w, h, seed) in enumerate(trace):
            while time.perf_counter() - t0 < ta:
                for (tag, st, l) in hvx.hvx_server_poll(s):
                    lat.append(l)
            key = (kind, w, h)
            if device:
                src, dst = dev_in[key][i % 4], dev_out[key][i % 8]
                hvx.hvx_server_submit_bound(s, templ[key], [
                    (timg[key][0], src.data_ptr(), src.stride(0) * src.element_size()),
                    (timg[key][1], dst.data_ptr(), dst.stride(0))], hvx.HVX_MEMORY_DEVICE, i)
            else:
                src, dst = host_in[key], outs[key][i % 8]
                hvx.hvx_server_submit(s, templ[key], src.data_ptr(), src.stride(0), dst.data_ptr(), dst.stride(0), i)
            px += w * h
        hvx.hvx_server_drain(s)
        t1 = time.perf_counter()
        for (tag, st, l) in hvx.hvx_server_poll(s, 4096):
            lat.append(l)
        steps = hvx.hvx_server_stats(s, 4)
        peak = hvx.hvx_server_stats(s, 2)
        hvx.hvx_release_server(s)
        lat = np.array(lat) * 1e3
        return {"p50_ms": round(float(np.percentile(lat, 50)), 3), "p99_ms": round(float(np.percentile(lat, 99)), 3),
                "mean_ms": round(float(lat.mean()), 3), "mpix_s": round(px / 1e6 / (t1 - t0), 1),
                "requests": len(lat), "device_steps": steps, "peak_device_bytes": peak}

    res = {"budget_bytes": budget, "max_slots": 16, "streams": 2, "requests_per_run": n_req}
    burst = [(0.0, k, w, h, sd) for (_, k, w, h, sd) in synth.serving_trace(1.0, n_req, seed=1)]
    mean_px = np.mean([w * h for (_, _, w, h, _) in burst])
    for device in (True, False):
        name = "device_resident" if device else "host_copy"
        # burst capacity: every request queued at once
        cap = run(hvx.HVX_SERVER_PLAIN, burst, device)
        ccap = run(hvx.HVX_SERVER_CONTINUOUS, burst, device)
        d = {"plain_burst": cap, "continuous_burst": ccap}
        rate_cap = cap["mpix_s"] * 1e6 / mean_px  # plain capacity in requests per second
        for frac in (0.5, 0.8, 0.95, 1.2):
            trace = synth.serving_trace(frac * rate_cap, n_req, seed=2)
            d["rate_%.2f" % frac] = {"rate_rps": round(frac * rate_cap, 1),
                                     "continuous": run(hvx.HVX_SERVER_CONTINUOUS, trace, device),
                                     "plain": run(hvx.HVX_SERVER_PLAIN, trace, device)}
        res[name] = d
        log("serving", name, json.dumps(d))
    for g in templ.values():
        hvx.hvx_release_graph(g)
    for (ih, oh) in timg.values():
        hvx.hvx_release_image(ih)
        hvx.hvx_release_image(oh)
    return res


def copy_calibration(torch, nbytes=1 << 30):
    """A plain device copy of known size: its FETCH_SIZE / WRITE_SIZE counter
    readings calibrate the HBM traffic counters of the other kernels."""
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1)
    torch.cuda.synchronize()
    ms, _ = time_region(torch, lambda: b.copy_(a), 5, 1)
    del a, b
    torch.cuda.empty_cache()
    return {"bytes": 2 * nbytes, "ms": round(ms, 4), "gbs": round(2 * nbytes / (ms / 1e3) / 1e9, 1)}


def _cpu_model():
    """CPU model name as lscpu reports it (else /proc/cpuinfo)."""
    import subprocess
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_cores(job_share=16):
    """Cores this process may use: its CPU affinity, bounded by the cgroup's
    CPU quota when one is set, and by the host-core share a one-GPU job is
    given on the GPU machines (16).  Returns (cores, details)."""
    aff = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    quota = None
    try:
        q, per = open("/sys/fs/cgroup/cpu.max").read().split()[:2]
        if q != "max":
            quota = max(1, int(int(q) / int(per)))
    except (OSError, ValueError):
        pass
    cores = min(aff, quota or aff, job_share)
    return max(1, cores), {"nproc": aff, "os_cpu_count": os.cpu_count(), "cgroup_cpu_quota": quota,
                           "job_core_share": job_share}


def cpu_baseline(w, h, budget_s=20.0):
    """The node-by-node C oracle on the headline graph, Gaussian3x3 ->
    Sobel3x3 -> {Magnitude -> Threshold(100), Phase} with REPLICATE borders
    and both U8 outputs: one thread, then one frame per thread on every core
    this job may use (each thread runs the unchanged oracle on its own frame,
    so the threaded figure is plain throughput scaling, no reblocking).  The
    edge map alone (no Phase) is timed the same way and reported beside it."""
    import concurrent.futures as cf

    import oracle
    import synth

    def edge_phase(img):
        gx, gy = oracle.sobel3x3(oracle.gaussian3x3(img))
        return oracle.threshold(oracle.magnitude(gx, gy), 100), oracle.phase(gx, gy)

    def edge_only(img):
        gx, gy = oracle.sobel3x3(oracle.gaussian3x3(img))
        return oracle.threshold(oracle.magnitude(gx, gy), 100)

    threads, cores_info = host_cores()
    imgs = [synth.edge_image(w, h, seed=i) for i in range(threads)]

    def rate(fn, budget):
        fn(imgs[0])  # build + page in
        t0 = time.perf_counter()
        n1 = 0
        while n1 < 8 and (n1 < 2 or time.perf_counter() - t0 < budget / 3):
            fn(imgs[0])
            n1 += 1
        dt1 = time.perf_counter() - t0
        stop = time.perf_counter() + budget * 2 / 3

        def worker(i):
            k = 0
            while True:
                fn(imgs[i])
                k += 1
                if time.perf_counter() > stop:
                    return k

        t0 = time.perf_counter()
        with cf.ThreadPoolExecutor(threads) as ex:
            nt = sum(ex.map(worker, range(threads)))
        dtt = time.perf_counter() - t0
        return n1, dt1, nt, dtt

    n1, dt1, nt, dtt = rate(edge_phase, budget_s * 0.6)
    e1, edt1, et, edtt = rate(edge_only, budget_s * 0.4)
    mp = w * h / 1e6
    model = _cpu_model()
    return dict(value=round(nt * mp / dtt, 2), unit="MPix/s", cores=threads, kind="oracle",
                single_thread_value=round(n1 * mp / dt1, 2),
                graph="Gaussian3x3->Sobel3x3->{Magnitude->Threshold(100), Phase}",
                edge_only={"value": round(et * mp / edtt, 2), "single_thread_value": round(e1 * mp / edt1, 2),
                           "graph": "Gaussian3x3->Sobel3x3->Magnitude->Threshold(100)"},
                cpu_model=model, host=cores_info,
                sample="%dx%d frames of the headline graph Gaussian3x3->Sobel3x3->{Magnitude->Threshold(100), "
                       "Phase} (REPLICATE, both U8 outputs) through the node-by-node C oracle: %d frames on %d "
                       "threads in %.1f s (one frame per thread); single thread %d frames in %.1f s; CPU %s"
                       % (w, h, nt, threads, dtt, n1, dt1, model))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--frames", type=int, default=64)
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--only", default=None,
                    help="comma-separated names of extra measurements (%s) to run alone, without the headline "
                         "(profiling runs)" % ", ".join(EXTRAS))
    ap.add_argument("--extra-rows", type=int, default=None,
                    help="with --only: pin the batches to this many rows per work item, direct launch (no tuning)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--rows", type=int, default=None,
                    help="pin the headline batch to this many rows per work item (default: tune)")
    ap.add_argument("--mode", choices=("auto", "direct", "persistent"), default="auto",
                    help="headline launch mode (default: time both, keep the faster)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only (the library has no multi-GPU path: images and requests shard with "
              "no exchange); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2008_11476_amd as hvx
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    ctx = hvx.hvx_context_create(0)
    # a stream of our own (default priority): the null stream cannot be
    # captured, so batches would run as plain launches there
    work = torch.cuda.Stream()
    with torch.cuda.stream(work):
        run(args, torch, hvx, ctx)
    hvx.hvx_context_release(ctx)


def run(args, torch, hvx, ctx):
    W, H = 3840, 2160
    copy_ref = copy_calibration(torch)  # also the known-size copy that calibrates the traffic counters
    log("plain device copy:", copy_ref)
    if args.only:
        names = args.only.split(",")
        bad = [n for n in names if n not in EXTRAS]
        if bad:
            print("unknown measurement(s): %s" % ", ".join(bad), file=sys.stderr)
            sys.exit(2)
        print(json.dumps(extras(hvx, torch, ctx, only=names, rows=args.extra_rows)), flush=True)
        return
    log("edge+phase graph: %d x %dx%d frames per step, %d steps" % (args.frames, W, H, args.steps))
    modes = ("persistent", "direct") if args.mode == "auto" else (args.mode,)
    r = edge_batch(hvx, torch, ctx, W, H, args.frames, args.steps, args.warmup, phase=True, rows=args.rows,
                   modes=modes)
    ms = r["ms"]
    kernel = "hvx::k_batch_direct<8>" if r["mode"] == "direct" else "hvx::k_batch<8>"
    # HBM bytes per launch from the committed FETCH_SIZE / WRITE_SIZE counter
    # summary (one entry per profiled rows-per-item shape), used only while it
    # matches the kernel sources and the tuned launch shape
    traffic = None
    tfile = os.path.join(ROOT, "profiles", "edge_phase_4k_batch_traffic.json")
    rows_key = str(r["per_mode"]["rows_per_item"])
    if os.path.exists(tfile):
        t = json.load(open(tfile))
        if t.get("kernel_hash") == kernel_source_hash() and t.get("kernel") == kernel:
            traffic = t.get("shapes", {}).get(rows_key, {}).get("bytes_per_launch")
    # VALU instructions per launch from the committed SQ counter summary (same
    # kernel sources and launch shape only): the share of the machine's VALU
    # issue slots the timed launches used, 1024 SIMDs x one wave64
    # instruction per 4 cycles at 2.4 GHz
    valu_frac = None
    vfile = os.path.join(ROOT, "profiles", "edge_phase_4k_batch_valu.json")
    if os.path.exists(vfile):
        v = json.load(open(vfile))
        insts = None
        if v.get("kernel_hash") == kernel_source_hash() and v.get("kernel") == kernel:
            insts = v.get("shapes", {}).get(rows_key, {}).get("valu_insts_per_launch")
        if insts:
            slots = VALU_SIMDS * (ms * 1e-3) * CLOCK_HZ / 4
            valu_frac = round(insts / slots, 4)
    out = {
        "metric": "fused-graph MPix/s + % HBM peak (4K Sobel); served p50/p99 latency vs plain",
        "value": round(r["mpix_s"], 1),
        "unit": "MPix/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic (seeded uniform U8 + 8 filled rectangles)",
        "config": {"workload": "sobel_edge_phase_4k_batch64",
                   "graph": "Gaussian3x3->Sobel3x3->{Magnitude->Threshold(100), Phase}",
                   "border": "replicate", "outputs": "edge map U8 + phase U8", "width": W, "height": H, "frames_per_step": args.frames,
                   "rows_per_item": r["per_mode"]["rows_per_item"],
                   "launch": "%s batch kernel, one launch per step" % r["mode"],
                   "batch_mode_ms": r["per_mode"]},
        "roofline": {"bound": "hbm", "achieved": round(r["gbs"], 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(r["gbs"] / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "kernel": kernel, "work_items": r["per_mode"]["work_items"],
                     "alg_bytes_per_launch": r["alg_bytes"],
                     "avg_launch_ms": round(ms, 4), "plain_copy_gbs": copy_ref["gbs"],
                     "valu_issue_frac": valu_frac},
    }
    log("headline (edge+phase): %.1f MPix/s, %.1f GB/s (%.1f%% of peak), %.3f ms/step, host %.3f ms/step" % (
        r["mpix_s"], r["gbs"], 100 * r["gbs"] / HBM_PEAK_GBS, ms, r["ms_host"]))
    if not args.no_extras:
        try:
            out["extras"] = extras(hvx, torch, ctx)
        except Exception as e:  # context numbers must never cost the headline
            import traceback
            traceback.print_exc()
            out["extras"] = {"error": repr(e)}
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(W, H)
        log("cpu baseline:", out["cpu_baseline"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
