"""GPU tests of batched execution (one kernel launch over many graphs,
replayed from a captured HIP graph) and of the serving loop: every result
must equal the same graph run alone, and the oracle."""
import time

import numpy as np
import pytest

import oracle
import paper_2008_11476_amd as hvx
import synth
from tests import graphspec as gs
from tests.gpu_util import compare, device_image, log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    c = hvx.hvx_context_create(0)
    yield c
    hvx.hvx_context_release(c)


def _mixed_specs():
    rng = np.random.default_rng(7)
    specs = []
    kinds = ["edge", "edge_phase", "corner", "gauss5", "uyvy", "generic", "unfused_edge"]
    for i in range(21):
        kind = kinds[i % len(kinds)]
        w = int(rng.integers(1, 2100)) if kind != "uyvy" else 2 * int(rng.integers(1, 1000))
        h = int(rng.integers(1, 300))
        if kind == "edge":
            specs.append((kind, gs.edge_spec(synth.edge_image(w, h, seed=i))))
        elif kind == "edge_phase":
            specs.append((kind, gs.edge_spec(synth.edge_image(w, h, seed=i), phase=True,
                                             b1=("constant", 9))))
        elif kind == "corner":
            specs.append((kind, gs.corner_spec(synth.corner_image(w, h, seed=i))))
        elif kind == "gauss5":
            specs.append((kind, gs.gauss5_spec(synth.edge_image(w, h, seed=i), ("constant", 3))))
        elif kind == "uyvy":
            specs.append((kind, gs.uyvy_gauss5_spec(synth.uyvy_image(w, h, seed=i))))
        elif kind == "generic":
            img = synth.edge_image(w, h, seed=i)
            specs.append((kind, gs.Spec([gs.N("box3x3", ["in"], ["b"]),
                                         gs.N("add", ["in", "b"], ["out"], params={"policy": "wrap"})],
                                        {"in": img}, {"out": np.uint8})))
        else:
            specs.append((kind, gs.edge_spec(synth.edge_image(w, h, seed=i))))
    return specs


def _build(ctx, spec, fusion=True):
    """Device images (random padding) + a verified graph; returns graph and
    {output name: (tensor, width)}."""
    imgs, keep, outs = {}, [], {}
    for name, arr in spec.inputs.items():
        df = hvx.HVX_DF_UYVY if name in spec.uyvy else gs.DF_OF_DTYPE[arr.dtype]
        im, t = device_image(ctx, arr, df, seed=3)
        imgs[name] = im
        keep.append(t)
        h = arr.shape[0]
        w = arr.shape[1] // 2 if df == hvx.HVX_DF_UYVY else arr.shape[1]
    for name, dt in spec.outputs.items():
        im, t = device_image(ctx, np.zeros((h, w), np.dtype(dt)), gs.DF_OF_DTYPE[np.dtype(dt)], seed=4)
        imgs[name] = im
        outs[name] = (t, w)
    g, _, _ = gs.build_hvx(spec, ctx, imgs)
    hvx.hvx_graph_set_option(g, hvx.HVX_OPT_FUSION, int(fusion))
    hvx.hvx_graph_verify(g, ctx=ctx)
    return g, outs, keep, imgs


def _read(outs):
    return {k: t.cpu().numpy()[:, :w] for k, (t, w) in outs.items()}


@pytest.mark.parametrize("persistent", [1, 0])
def test_batch_equals_alone_and_oracle(ctx, persistent):
    import torch
    specs = _mixed_specs()
    built = []
    for kind, spec in specs:
        g, outs, keep, imgs = _build(ctx, spec, fusion=(kind != "unfused_edge"))
        built.append((kind, spec, g, outs, keep))
    # alone
    alone = []
    for kind, spec, g, outs, keep in built:
        log("alone %s" % kind)
        hvx.hvx_graph_process(g, ctx=ctx)
        alone.append(_read(outs))
        for t, _ in outs.values():
            t.fill_(0x5A)
    torch.cuda.synchronize()
    b = hvx.hvx_batch_create(ctx, [x[2] for x in built])
    hvx.hvx_batch_set_option(b, hvx.HVX_BATCH_PERSISTENT, persistent)
    assert hvx.hvx_batch_query(b, hvx.HVX_QUERY_NUM_KERNELS) >= 2  # the batch launch + separate graphs
    side = torch.cuda.Stream()  # capturable (the null stream is not)
    stream = side.cuda_stream
    for rep in range(3):  # capture, then replays with eager work in between
        log("batch replay %d" % rep)
        hvx.hvx_batch_schedule(b, stream, ctx=ctx)
        torch.cuda.synchronize()
        for (kind, spec, g, outs, keep), ref in zip(built, alone):
            got = _read(outs)
            for name in got:
                assert np.array_equal(got[name], ref[name]), (kind, name, rep)
            for t, _ in outs.values():
                t.fill_(rep)
        torch.cuda.synchronize()
    # against the oracle too
    for (kind, spec, g, outs, keep), ref in zip(built, alone):
        env = spec.run_oracle()
        compare(spec, ref, env, phase_names=("ph",), corner=(kind == "corner"))
    hvx.hvx_release_batch(b)


def test_batch_rows_option(ctx):
    """Pinned rows per work item (any value, ragged bands included) give the
    oracle's result in both launch modes; out-of-range values are rejected."""
    import torch
    w, h = 2100, 77
    a = synth.edge_image(w, h, seed=3)
    spec = gs.edge_spec(a, phase=True)
    env = spec.run_oracle()
    g, outs, keep, imgs = _build(ctx, spec)
    b = hvx.hvx_batch_create(ctx, [g])
    side = torch.cuda.Stream()  # capturable (the null stream is not)
    stream = side.cuda_stream
    for rows in (1, 5, 32, 200):
        for pers in (1, 0):
            log("batch rows=%d persistent=%d" % (rows, pers))
            hvx.hvx_batch_set_option(b, hvx.HVX_BATCH_ROWS, rows, ctx=ctx)
            hvx.hvx_batch_set_option(b, hvx.HVX_BATCH_PERSISTENT, pers, ctx=ctx)
            assert hvx.hvx_batch_query(b, hvx.HVX_QUERY_ROWS_PER_ITEM) == rows
            for t, _ in outs.values():
                t.fill_(0x5A)
            torch.cuda.synchronize()
            hvx.hvx_batch_schedule(b, stream, ctx=ctx)
            torch.cuda.synchronize()
            compare(spec, _read(outs), env, phase_names=("ph",))
    for bad in (-1, 65536):
        with pytest.raises(hvx.HvxError):
            hvx.hvx_batch_set_option(b, hvx.HVX_BATCH_ROWS, bad, ctx=ctx)
    hvx.hvx_release_batch(b)


@pytest.mark.parametrize("kind", ["edge", "edge_constant", "edge_wide", "edge_phase_constant", "gauss5", "uyvy_gauss5",
                                  "corner"])
def test_batch_short_bands_every_stream(ctx, kind):
    """Bands of 1 to 9 rows (shorter than the row queue and its prologue),
    on a frame whose height leaves a ragged last band, through each fused
    stream in both launch modes: the explicit memory waits of the row queues
    have their start and end cases here.  The edge stream without Phase runs
    odd bands bottom-up; its ragged last band is odd for 4, 5 and 7 rows."""
    import torch
    w, h = 1100, 37
    if kind == "edge":
        spec = gs.edge_spec(synth.edge_image(w, h, seed=21))
    elif kind == "edge_constant":
        spec = gs.edge_spec(synth.edge_image(w, h, seed=26), b0=("constant", 9), b1=("constant", 0))
    elif kind == "edge_wide":  # threshold 200: the 32-bit magnitude test
        spec = gs.edge_spec(synth.edge_image(w, h, seed=27), b0=("constant", 250), thresh=200)
    elif kind == "edge_phase_constant":
        spec = gs.edge_spec(synth.edge_image(w, h, seed=22), phase=True, b0=("constant", 9), b1=("constant", 0))
    elif kind == "gauss5":
        spec = gs.gauss5_spec(synth.edge_image(w, h, seed=23), b=("constant", 200))
    elif kind == "uyvy_gauss5":
        spec = gs.uyvy_gauss5_spec(synth.uyvy_image(w, h, seed=24))
    else:
        spec = gs.corner_spec(synth.corner_image(w, h, seed=25))
    env = spec.run_oracle()
    g, outs, keep, imgs = _build(ctx, spec)
    b = hvx.hvx_batch_create(ctx, [g])
    side = torch.cuda.Stream()
    stream = side.cuda_stream
    for rows in (1, 2, 3, 4, 5, 6, 7, 9):
        for pers in (0, 1):
            log("short bands %s rows=%d persistent=%d" % (kind, rows, pers))
            hvx.hvx_batch_set_option(b, hvx.HVX_BATCH_ROWS, rows, ctx=ctx)
            hvx.hvx_batch_set_option(b, hvx.HVX_BATCH_PERSISTENT, pers, ctx=ctx)
            for t, _ in outs.values():
                t.fill_(0x5A)
            torch.cuda.synchronize()
            hvx.hvx_batch_schedule(b, stream, ctx=ctx)
            torch.cuda.synchronize()
            compare(spec, _read(outs), env, phase_names=("ph",), corner=(kind == "corner"))
    hvx.hvx_release_batch(b)
    hvx.hvx_release_graph(g)


def test_batch_refresh_after_swap(ctx):
    import torch
    w, h = 1500, 90
    a = synth.edge_image(w, h, seed=1)
    bimg = synth.edge_image(w, h, seed=2)
    spec = gs.edge_spec(a, phase=True)
    g, outs, keep, imgs = _build(ctx, spec)
    other, t2 = device_image(ctx, bimg, hvx.HVX_DF_U8, seed=9)
    b = hvx.hvx_batch_create(ctx, [g])
    side = torch.cuda.Stream()  # capturable (the null stream is not)
    stream = side.cuda_stream
    hvx.hvx_batch_schedule(b, stream, ctx=ctx)
    torch.cuda.synchronize()
    compare(spec, _read(outs), spec.run_oracle(), phase_names=("ph",))
    hvx.hvx_image_swap_ptr(imgs["in"], t2.data_ptr(), t2.stride(0), ctx=ctx)
    hvx.hvx_batch_refresh(b, ctx=ctx)
    hvx.hvx_batch_schedule(b, stream, ctx=ctx)
    torch.cuda.synchronize()
    spec2 = gs.edge_spec(bimg, phase=True)
    compare(spec2, _read(outs), spec2.run_oracle(), phase_names=("ph",))
    hvx.hvx_release_batch(b)
    # the one-shot form
    hvx.hvx_process_batch(ctx, [g], stream)
    compare(spec2, _read(outs), spec2.run_oracle(), phase_names=("ph",))


def _templates(ctx, sizes):
    """Verified templates for the three served kinds at each size."""
    out = {}
    keep = []
    for (w, h) in sizes:
        for kind in ("sobel_edge", "harris", "uyvy_gauss5"):
            if kind == "uyvy_gauss5":
                spec = gs.uyvy_gauss5_spec(synth.uyvy_image(w, h, seed=w))
            elif kind == "harris":
                spec = gs.corner_spec(synth.corner_image(w, h, seed=w))
            else:
                spec = gs.edge_spec(synth.edge_image(w, h, seed=w))
            g, outs, k, imgs = _build(ctx, spec)
            keep.append((outs, k))
            out[(kind, w, h)] = g
    return out, keep


def _host_frames(kind, w, h, seed):
    if kind == "uyvy_gauss5":
        f = synth.uyvy_image(w, h, seed=seed)
        spec = gs.uyvy_gauss5_spec(f)
    elif kind == "harris":
        f = synth.corner_image(w, h, seed=seed)
        spec = gs.corner_spec(f)
    else:
        f = synth.edge_image(w, h, seed=seed)
        spec = gs.edge_spec(f)
    return f, spec


@pytest.mark.parametrize("mode", [hvx.HVX_SERVER_CONTINUOUS, hvx.HVX_SERVER_PLAIN])
def test_server_results_alone_equals_mix(ctx, mode):
    import torch
    sizes = [(64, 48), (322, 101), (640, 480)]
    templ, keep = _templates(ctx, sizes)
    budget = 3 << 20  # binds: a 640x480 request needs ~0.6 MB
    s = hvx.hvx_server_create(ctx, mode, budget, 4, 2)
    reqs = {}
    rng = np.random.default_rng(3)
    for tag in range(36):
        kind = ("sobel_edge", "harris", "uyvy_gauss5")[tag % 3]
        w, h = sizes[int(rng.integers(0, len(sizes)))]
        f, spec = _host_frames(kind, w, h, seed=100 + tag)
        src = torch.from_numpy(np.ascontiguousarray(f)).pin_memory()
        dst = torch.full((h, w), 7, dtype=torch.uint8).pin_memory()
        reqs[tag] = (kind, spec, src, dst)
        if tag == 13:
            hvx.hvx_server_inject_failure(s, tag)
        log("submit %d %s %dx%d" % (tag, kind, w, h))
        hvx.hvx_server_submit(s, templ[(kind, w, h)], src.data_ptr(), src.stride(0), dst.data_ptr(),
                              dst.stride(0), tag, ctx=ctx)
        if tag % 5 == 0:
            time.sleep(0.002)
    hvx.hvx_server_drain(s, ctx=ctx)
    done = hvx.hvx_server_poll(s, 1000, ctx=ctx)
    assert sorted(t for t, _, _ in done) == list(range(36))
    assert hvx.hvx_server_stats(s, 2) <= budget  # peak device bytes
    assert hvx.hvx_server_stats(s, 5) == 0  # everything released
    for tag, st, lat in done:
        kind, spec, src, dst = reqs[tag]
        if tag == 13:
            assert st == hvx.HVX_ERROR_DEVICE
            continue
        assert st == 0 and lat > 0
        env = spec.run_oracle()
        compare(spec, {"out": dst.numpy()}, env, corner=(kind == "harris"))
    if mode == hvx.HVX_SERVER_CONTINUOUS:
        assert hvx.hvx_server_stats(s, 4) <= 36  # requests were packed into shared device steps
    hvx.hvx_release_server(s)


@pytest.mark.parametrize("mode", [hvx.HVX_SERVER_CONTINUOUS, hvx.HVX_SERVER_PLAIN])
def test_server_configured_sizes(ctx, mode):
    """The serving workload's own sizes, 640x480 to 3840x2160, for the three
    served graphs, under a budget that binds (a 4K UYVY request holds 24.9 MB,
    the budget 40 MiB): every result against the oracle, then every request
    served again alone, byte-equal to its result in the mix."""
    import torch
    sizes = list(synth.SERVE_SIZES)
    templ, keep = _templates(ctx, sizes)
    budget = 40 << 20
    reqs = {}
    tag = 0
    for (w, h) in sizes:
        for kind in synth.SERVE_TYPES:
            for rep in range(2):
                f, spec = _host_frames(kind, w, h, seed=200 + tag)
                src = torch.from_numpy(np.ascontiguousarray(f)).pin_memory()
                reqs[tag] = (kind, w, h, spec, src)
                tag += 1
    order = list(np.random.default_rng(11).permutation(len(reqs)))

    def serve(tags, drain_each):
        s = hvx.hvx_server_create(ctx, mode, budget, 8, 2)
        dst = {}
        for t in tags:
            kind, w, h, spec, src = reqs[t]
            dst[t] = torch.full((h, w), 7, dtype=torch.uint8).pin_memory()
            hvx.hvx_server_submit(s, templ[(kind, w, h)], src.data_ptr(), src.stride(0), dst[t].data_ptr(),
                                  dst[t].stride(0), t, ctx=ctx)
            if drain_each:
                hvx.hvx_server_drain(s, ctx=ctx)
        hvx.hvx_server_drain(s, ctx=ctx)
        done = hvx.hvx_server_poll(s, 1000, ctx=ctx)
        assert sorted(t for t, _, _ in done) == sorted(tags)
        assert all(st == 0 for _, st, _ in done)
        assert hvx.hvx_server_stats(s, 2) <= budget
        hvx.hvx_release_server(s)
        return dst

    log("serving %d requests at the configured sizes, mode %d" % (len(order), mode))
    mix = serve(order, False)
    for t in sorted(reqs):
        kind, w, h, spec, src = reqs[t]
        log("served %d %s %dx%d vs oracle" % (t, kind, w, h))
        compare(spec, {"out": mix[t].numpy()}, spec.run_oracle(), corner=(kind == "harris"))
    alone = serve(sorted(reqs), True)
    for t in sorted(reqs):
        assert torch.equal(alone[t], mix[t]), t


def test_server_limits(ctx):
    with pytest.raises(hvx.HvxError) as e:
        hvx.hvx_server_create(ctx, hvx.HVX_SERVER_CONTINUOUS, 0, 4, 2)
    assert e.value.status == hvx.HVX_ERROR_NO_MEMORY
    templ, keep = _templates(ctx, [(640, 480)])
    s = hvx.hvx_server_create(ctx, hvx.HVX_SERVER_CONTINUOUS, 1 << 16, 4, 2)
    import torch
    src = torch.zeros((480, 640), dtype=torch.uint8).pin_memory()
    dst = torch.zeros((480, 640), dtype=torch.uint8).pin_memory()
    with pytest.raises(hvx.HvxError) as e:
        hvx.hvx_server_submit(s, templ[("sobel_edge", 640, 480)], src.data_ptr(), 640, dst.data_ptr(), 640, 1,
                              ctx=ctx)
    assert e.value.status == hvx.HVX_ERROR_NO_MEMORY
    hvx.hvx_release_server(s)


def test_server_rejects_unservable_templates(ctx):
    """The one-image call refuses a template with two outputs (the edge
    graph with its Phase output: hvx_server_submit_bound serves it), and no
    call serves a template whose results are global-operator buffers."""
    import torch
    w, h = 256, 64
    img = synth.edge_image(w, h, seed=2)
    s = hvx.hvx_server_create(ctx, hvx.HVX_SERVER_CONTINUOUS, 64 << 20, 4, 2)
    src = torch.zeros((h, w), dtype=torch.uint8).pin_memory()
    dst = torch.zeros((h, w), dtype=torch.uint8).pin_memory()
    g, outs, keep, imgs = _build(ctx, gs.edge_spec(img, phase=True))
    with pytest.raises(hvx.HvxError) as e:
        hvx.hvx_server_submit(s, g, src.data_ptr(), w, dst.data_ptr(), w, 7, ctx=ctx)
    assert e.value.status == hvx.HVX_ERROR_NOT_SUPPORTED
    # an image left unbound, or bound twice
    with pytest.raises(hvx.HvxError) as e:
        hvx.hvx_server_submit_bound(s, g, [(imgs["in"], src.data_ptr(), w)], hvx.HVX_MEMORY_HOST, 8, ctx=ctx)
    assert e.value.status == hvx.HVX_ERROR_INVALID_PARAMETERS
    with pytest.raises(hvx.HvxError) as e:
        hvx.hvx_server_submit_bound(s, g, [(imgs["in"], src.data_ptr(), w)] * 2 + [
            (imgs["out"], dst.data_ptr(), w), (imgs["ph"], dst.data_ptr(), w)], hvx.HVX_MEMORY_HOST, 9, ctx=ctx)
    assert e.value.status == hvx.HVX_ERROR_INVALID_PARAMETERS
    hvx.hvx_release_graph(g)
    buf = torch.zeros(1024, dtype=torch.uint8, device="cuda")
    spec = gs.Spec([gs.N("gaussian3x3", ["in"], ["out"]), gs.N("histogram", ["out"], ["hist"], params={"bins": 16})],
                   {"in": img}, {"out": np.uint8}, buffers={"hist": 1024})
    im, t = device_image(ctx, img, hvx.HVX_DF_U8)
    om, t2 = device_image(ctx, np.zeros((h, w), np.uint8), hvx.HVX_DF_U8)
    gh, _, _ = gs.build_hvx(spec, ctx, {"in": im, "out": om, "hist": hvx.hvx_buffer_from_ptr(ctx, buf.data_ptr(), 1024)})
    with pytest.raises(hvx.HvxError) as e:
        hvx.hvx_server_submit(s, gh, src.data_ptr(), w, dst.data_ptr(), w, 10, ctx=ctx)
    assert e.value.status == hvx.HVX_ERROR_NOT_SUPPORTED
    hvx.hvx_release_graph(gh)
    hvx.hvx_release_server(s)


def _bound_specs(w, h, seed):
    """Templates served through bindings: a two-output strip kernel, a fused
    generic kernel, and two plans of two kernels each (EqualizeHist before
    and after a Gaussian; the second keeps the Gaussian in a scratch block of
    the request's own)."""
    img = synth.edge_image(w, h, seed=seed)
    return {
        "edge_phase": gs.edge_spec(img, phase=True),
        "generic": gs.Spec([gs.N("box3x3", ["in"], ["b"]), gs.N("add", ["in", "b"], ["out"], params={"policy": "wrap"})],
                           {"in": img}, {"out": np.uint8}),
        "eqhist_gauss": gs.Spec([gs.N("equalize_hist", ["in"], ["e"]), gs.N("gaussian3x3", ["e"], ["out"])],
                                {"in": img}, {"out": np.uint8}),
        "gauss_eqhist": gs.Spec([gs.N("gaussian3x3", ["in"], ["g"]), gs.N("equalize_hist", ["g"], ["out"])],
                                {"in": img}, {"out": np.uint8}),
    }


@pytest.mark.parametrize("mode", [hvx.HVX_SERVER_CONTINUOUS, hvx.HVX_SERVER_PLAIN])
def test_server_bound_requests_device_and_host(ctx, mode):
    """Requests bound to device-resident frames (run in place) and to host
    frames (copied), over templates with two outputs, generic kernels and
    plans with intermediates in per-request scratch, interleaved under a
    budget that binds: every output equals the oracle's for its own input."""
    import torch
    sizes = [(64, 48), (640, 480)]
    templ = {}
    for (w, h) in sizes:
        for kind, spec in _bound_specs(w, h, seed=1).items():
            g, outs, keep, imgs = _build(ctx, spec)
            templ[(kind, w, h)] = (g, imgs, keep, outs)
    budget = 4 << 20
    s = hvx.hvx_server_create(ctx, mode, budget, 6, 2)
    reqs = {}
    rng = np.random.default_rng(11)
    for tag in range(32):
        kind = ("edge_phase", "generic", "eqhist_gauss", "gauss_eqhist")[tag % 4]
        w, h = sizes[int(rng.integers(0, len(sizes)))]
        device = bool(rng.integers(0, 2))
        spec = _bound_specs(w, h, seed=200 + tag)[kind]
        g, imgs, _, _ = templ[(kind, w, h)]
        bind, held = [], {}
        for name, arr in spec.inputs.items():
            if device:
                buf, view = hvx.alloc_image(h, w, hvx.HVX_DF_U8)
                view.copy_(torch.from_numpy(arr))
                held[name] = view
                bind.append((imgs[name], view.data_ptr(), view.stride(0)))
            else:
                t = torch.from_numpy(np.ascontiguousarray(arr)).pin_memory()
                held[name] = t
                bind.append((imgs[name], t.data_ptr(), t.stride(0)))
        for name in spec.outputs:
            if device:
                buf, view = hvx.alloc_image(h, w, hvx.HVX_DF_U8)
                view.fill_(7)
                held[name] = view
                bind.append((imgs[name], view.data_ptr(), view.stride(0)))
            else:
                t = torch.full((h, w), 7, dtype=torch.uint8).pin_memory()
                held[name] = t
                bind.append((imgs[name], t.data_ptr(), t.stride(0)))
        torch.cuda.synchronize()
        reqs[tag] = (kind, spec, held)
        log("submit %d %s %dx%d %s" % (tag, kind, w, h, "device" if device else "host"))
        hvx.hvx_server_submit_bound(s, g, bind, hvx.HVX_MEMORY_DEVICE if device else hvx.HVX_MEMORY_HOST, tag, ctx=ctx)
        if tag % 6 == 0:
            time.sleep(0.002)
    hvx.hvx_server_drain(s, ctx=ctx)
    done = hvx.hvx_server_poll(s, 1000, ctx=ctx)
    assert sorted(t for t, _, _ in done) == list(range(32))
    assert hvx.hvx_server_stats(s, 2) <= budget
    assert hvx.hvx_server_stats(s, 5) == 0
    for tag, st, lat in done:
        kind, spec, held = reqs[tag]
        assert st == 0 and lat > 0, (tag, st)
        env = spec.run_oracle()
        got = {name: held[name].cpu().numpy() for name in spec.outputs}
        compare(spec, got, env, phase_names=("ph",))
    hvx.hvx_release_server(s)
    for (g, imgs, keep, outs) in templ.values():
        hvx.hvx_release_graph(g)


def test_templates_outlive_their_server():
    """Templates a server ran requests on are waited on and released, with
    their context, after the server and its streams are gone: a run on the
    server's stream is the server's to wait for, not the graph's."""
    import torch
    c = hvx.hvx_context_create(0)
    spec = _bound_specs(64, 48, seed=3)["generic"]
    g, outs, keep, imgs = _build(c, spec)
    s = hvx.hvx_server_create(c, hvx.HVX_SERVER_CONTINUOUS, 1 << 22, 4, 2)
    held, bind = {}, []
    for name, arr in spec.inputs.items():
        buf, view = hvx.alloc_image(48, 64, hvx.HVX_DF_U8)
        view.copy_(torch.from_numpy(arr))
        held[name] = view
        bind.append((imgs[name], view.data_ptr(), view.stride(0)))
    for name in spec.outputs:
        buf, view = hvx.alloc_image(48, 64, hvx.HVX_DF_U8)
        held[name] = view
        bind.append((imgs[name], view.data_ptr(), view.stride(0)))
    torch.cuda.synchronize()
    log("template outlives server: submit")
    hvx.hvx_server_submit_bound(s, g, bind, hvx.HVX_MEMORY_DEVICE, 1, ctx=c)
    hvx.hvx_server_drain(s, ctx=c)
    done = hvx.hvx_server_poll(s, 8, ctx=c)
    assert [t for t, _, _ in done] == [1] and done[0][1] == 0
    compare(spec, {n: held[n].cpu().numpy() for n in spec.outputs}, spec.run_oracle())
    hvx.hvx_release_server(s)
    hvx.hvx_graph_wait(g, ctx=c)
    hvx.hvx_context_release(c)


@pytest.mark.parametrize("use_graph", [1, 0])
def test_batch_runs_generated_kernels_once_per_kernel(ctx, use_graph):
    """Graphs whose plan is one generated kernel share a launch with the
    other graphs of that kernel (any sizes): four Unsharp graphs, two FChain
    graphs and two point chains run as three launches, a lone Tomasi graph as
    its own, the edge graph in the batch launch; outputs equal each graph run
    alone and the oracle."""
    import torch
    from tests.test_gpu_codegen import _fchain, _point_chain, _tomasi
    from tests.test_gpu_custom import unsharp_spec
    specs = [("unsharp", unsharp_spec(synth.edge_image(w, h, seed=w))) for (w, h) in
             ((640, 480), (131, 29), (1, 1), (64, 48))]
    specs += [("fchain", _fchain(synth.edge_image(w, h, seed=h), ("replicate", 0))) for (w, h) in ((300, 77), (17, 5))]
    specs += [("point_chain", _point_chain(synth.uniform_u8(w, h, seed=3), synth.uniform_u8(w, h, seed=4)))
              for (w, h) in ((1029, 3), (66, 40))]
    specs += [("tomasi", _tomasi(synth.corner_image(129, 37, seed=1))), ("edge", gs.edge_spec(synth.edge_image(500, 60)))]
    built = []
    for kind, spec in specs:
        g, outs, keep, imgs = _build(ctx, spec)
        built.append((kind, spec, g, outs, keep))
    alone = []
    for kind, spec, g, outs, keep in built:
        hvx.hvx_graph_process(g, ctx=ctx)
        alone.append(_read(outs))
        for t, _ in outs.values():
            t.fill_(0x5A)
    torch.cuda.synchronize()
    b = hvx.hvx_batch_create(ctx, [x[2] for x in built])
    hvx.hvx_batch_set_option(b, hvx.HVX_BATCH_USE_GRAPH, use_graph)
    assert hvx.hvx_batch_query(b, hvx.HVX_QUERY_NUM_KERNELS) == 5
    side = torch.cuda.Stream()
    for rep in range(2):
        log("generated batch use_graph=%d rep %d" % (use_graph, rep))
        hvx.hvx_batch_schedule(b, side.cuda_stream, ctx=ctx)
        torch.cuda.synchronize()
        for (kind, spec, g, outs, keep), ref in zip(built, alone):
            got = _read(outs)
            for name in got:
                if got[name].dtype == np.float32:
                    assert np.array_equal(got[name].view(np.uint32), ref[name].view(np.uint32)), (kind, name, rep)
                else:
                    assert np.array_equal(got[name], ref[name]), (kind, name, rep)
            for t, _ in outs.values():
                t.fill_(rep + 1)
        torch.cuda.synchronize()
    for (kind, spec, g, outs, keep), ref in zip(built, alone):
        if kind == "tomasi":
            continue  # F32 response: its own test compares it within tolerance
        compare(spec, ref, spec.run_oracle(), phase_names=("ph",))
    hvx.hvx_release_batch(b)
    for x in built:
        hvx.hvx_release_graph(x[2])


def test_batch_runs_generated_chains_once_per_kernel(ctx, tmp_path):
    """Graphs whose plan is a chain of generated kernels (FChain cut at every
    value by a plan in the tune cache: three kernels) share one launch per
    kernel of the chain, in plan order, so each kernel still runs after the
    one it reads; outputs equal each graph run alone and the oracle."""
    import json
    import torch
    from tests.test_gpu_codegen import _fchain
    w, h = 300, 77
    # the plan key of this graph shape, from a tuned copy in its own context
    c1 = hvx.hvx_context_create(0)
    try:
        g0, outs0, keep0, imgs0 = _build(c1, _fchain(synth.edge_image(w, h, seed=1), ("replicate", 0)))
        hvx.hvx_graph_autotune(g0, torch.cuda.current_stream().cuda_stream, 1, ctx=c1)
        path = tmp_path / "tune.json"
        hvx.hvx_context_save_tune_cache(c1, str(path))
        hvx.hvx_release_graph(g0)
    finally:
        hvx.hvx_context_release(c1)
    keys = [k for k in json.loads(path.read_text()) if k.startswith("plan|")]
    assert len(keys) == 1, keys
    forced = tmp_path / "forced.json"
    forced.write_text(json.dumps({keys[0]: [0, 1, 1.0, list(range(64)), []]}))
    c2 = hvx.hvx_context_create(0)
    try:
        hvx.hvx_context_load_tune_cache(c2, str(forced))
        built = []
        for seed in (2, 3, 4):
            spec = _fchain(synth.edge_image(w, h, seed=seed), ("replicate", 0))
            g, outs, keep, imgs = _build(c2, spec)
            assert hvx.hvx_graph_query(g, hvx.HVX_QUERY_NUM_KERNELS) == 3
            assert hvx.hvx_graph_query(g, hvx.HVX_QUERY_NUM_GENERATED) == 3
            built.append((spec, g, outs, keep))
        alone = []
        for spec, g, outs, keep in built:
            hvx.hvx_graph_process(g, ctx=c2)
            alone.append(_read(outs))
            for t, _ in outs.values():
                t.fill_(0x5A)
        torch.cuda.synchronize()
        b = hvx.hvx_batch_create(c2, [x[1] for x in built])
        assert hvx.hvx_batch_query(b, hvx.HVX_QUERY_NUM_KERNELS) == 3
        for rep in range(2):
            log("generated chain batch rep %d" % rep)
            hvx.hvx_batch_schedule(b, torch.cuda.current_stream().cuda_stream, ctx=c2)
            torch.cuda.synchronize()
            for (spec, g, outs, keep), ref in zip(built, alone):
                got = _read(outs)
                for name in got:
                    assert np.array_equal(got[name], ref[name]), (name, rep)
                compare(spec, got, spec.run_oracle())
                for t, _ in outs.values():
                    t.fill_(rep + 1)
            torch.cuda.synchronize()
        hvx.hvx_release_batch(b)
        for x in built:
            hvx.hvx_release_graph(x[1])
    finally:
        hvx.hvx_context_release(c2)
