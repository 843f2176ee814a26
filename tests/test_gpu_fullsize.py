"""GPU parity at the workloads' full sizes, in the launch configuration the
benchmark times (tuned batch, persistent and direct modes, HIP-graph replay),
plus the F32 operators of the corner graph against the FP64 oracle.

Full-size outputs are checked against the oracle on sampled whole images (the
oracle finishes a 4K frame in well under a second); every image of a batch is
also compared between the two launch modes."""
import numpy as np
import pytest

import paper_2008_11476_amd as hvx
import synth
from tests import graphspec as gs
from tests.gpu_util import compare, device_image, log, run_spec

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = hvx.hvx_context_create(0)
    yield c
    hvx.hvx_context_release(c)


def _build_batch(ctx, specs):
    """Device images and verified graphs for a list of specs (one output each
    plus optional phase); returns (graphs, outputs, keep-alive list)."""
    graphs, outs, keep = [], [], []
    for i, spec in enumerate(specs):
        imgs = {}
        for name, arr in spec.inputs.items():
            df = hvx.HVX_DF_UYVY if name in spec.uyvy else gs.DF_OF_DTYPE[arr.dtype]
            im, t = device_image(ctx, arr, df, seed=i)
            imgs[name] = im
            keep.append(t)
            h, w = spec.shapes()[name]
        o = {}
        for name, dt in spec.outputs.items():
            im, t = device_image(ctx, np.zeros((h, w), np.dtype(dt)), gs.DF_OF_DTYPE[np.dtype(dt)], seed=i + 7)
            imgs[name] = im
            o[name] = (t, w)
        g, _, _ = gs.build_hvx(spec, ctx, imgs)
        hvx.hvx_graph_verify(g, ctx=ctx)
        graphs.append(g)
        outs.append(o)
    return graphs, outs, keep


def _run_modes(ctx, graphs, outs, check):
    """Tune the batch as the benchmark does, then run it in both launch modes
    (each captured and replayed twice, outputs poisoned in between); `check`
    gets the per-image outputs of the first mode, and the second mode must
    reproduce them byte for byte."""
    import torch
    side = torch.cuda.Stream()  # capturable (the null stream is not)
    stream = side.cuda_stream
    b = hvx.hvx_batch_create(ctx, graphs)
    hvx.hvx_batch_autotune(b, stream, 1, ctx=ctx)
    log("batch tuned: rows %d, %d work items" % (hvx.hvx_batch_query(b, hvx.HVX_QUERY_ROWS_PER_ITEM),
                                                  hvx.hvx_batch_query(b, hvx.HVX_QUERY_NUM_OPS)))
    first = None
    for persistent in (1, 0):
        hvx.hvx_batch_set_option(b, hvx.HVX_BATCH_PERSISTENT, persistent)
        for rep in range(2):
            for o in outs:
                for t, _ in o.values():
                    t.fill_(0x5A + rep)
            torch.cuda.synchronize()
            log("batch persistent=%d replay %d" % (persistent, rep))
            hvx.hvx_batch_schedule(b, stream, ctx=ctx)
            torch.cuda.synchronize()
            cur = [{k: t[:, :w].clone() for k, (t, w) in o.items()} for o in outs]
            if first is None:
                first = cur
                check(first)
            else:
                for i, (a, c) in enumerate(zip(first, cur)):
                    for k in a:
                        assert torch.equal(a[k], c[k]), (i, k, persistent, rep)
    hvx.hvx_release_batch(b)


def test_edge_4k_batch64_bench_launch(ctx):
    """64 distinct 3840x2160 frames, the benchmark's headline workload."""
    w, h, n = 3840, 2160, 64
    specs = [gs.edge_spec(synth.edge_image(w, h, seed=i)) for i in range(n)]
    graphs, outs, keep = _build_batch(ctx, specs)

    def check(res):
        for i in (0, 1, 31, 62, 63):
            log("4K frame %d vs oracle" % i)
            got = {k: v.cpu().numpy() for k, v in res[i].items()}
            compare(specs[i], got, specs[i].run_oracle())

    _run_modes(ctx, graphs, outs, check)
    for g in graphs:
        hvx.hvx_release_graph(g)


def _recipe_batch(ctx, w, h, n, phase=True, border=None):
    """The benchmark's frames on the device: frame i is seeded base
    synth.frame_recipe(i) XORed with its byte, outputs poisoned.  Returns
    (graphs, {output name: (view, width)} per frame, keep-alive list)."""
    import torch
    nb = min(n, 4)
    bases = [torch.from_numpy(synth.edge_image(w, h, seed=s)).cuda() for s in range(nb)]
    graphs, outs, keep = [], [], []
    for i in range(n):
        base, x = synth.frame_recipe(i, nb)
        ib, iv = hvx.alloc_image(h, w, hvx.HVX_DF_U8)
        iv.copy_(bases[base] ^ x)
        o = {}
        imgs = {"in": hvx.image_from_tensor(ctx, iv, hvx.HVX_DF_U8)}
        for name in (("out", "ph") if phase else ("out",)):
            ob, ov = hvx.alloc_image(h, w, hvx.HVX_DF_U8)
            ob.fill_(0x5A)
            imgs[name] = hvx.image_from_tensor(ctx, ov, hvx.HVX_DF_U8)
            o[name] = (ov, w)
            keep.append(ob)
        spec = gs.edge_spec(np.zeros((1, 1), np.uint8), phase=phase,
                            **({} if border is None else {"b0": border, "b1": border}))
        g, _, _ = gs.build_hvx(spec, ctx, imgs)
        hvx.hvx_graph_verify(g, ctx=ctx)
        graphs.append(g)
        outs.append(o)
        keep.append(ib)
    torch.cuda.synchronize()
    return graphs, outs, keep


def test_edge_phase_4k_batch64_headline(ctx):
    """The benchmarked workload itself: 64 distinct 3840x2160 frames built as
    the benchmark builds them, edge map + Phase, REPLICATE, in one direct
    batch launch of 45 rows per work item (the shape the tuner picks on
    MI355X), then in the shape the tuner picks here, in both launch modes.
    Sampled frames element by element against the oracle (edge map exact,
    Phase within one level circularly); every frame byte-equal across the
    launch shapes."""
    import torch
    w, h, n = 3840, 2160, 64
    graphs, outs, keep = _recipe_batch(ctx, w, h, n)
    side = torch.cuda.Stream()
    stream = side.cuda_stream
    b = hvx.hvx_batch_create(ctx, graphs)
    hvx.hvx_batch_set_option(b, hvx.HVX_BATCH_ROWS, 45, ctx=ctx)
    hvx.hvx_batch_set_option(b, hvx.HVX_BATCH_PERSISTENT, 0, ctx=ctx)
    assert hvx.hvx_batch_query(b, hvx.HVX_QUERY_NUM_KERNELS) == 1
    assert hvx.hvx_batch_query(b, hvx.HVX_QUERY_NUM_OPS) == n * 4 * 48  # 4 strips x 48 bands per frame
    log("headline: 64 x 4K edge+phase, rows 45, direct")
    hvx.hvx_batch_schedule(b, stream, ctx=ctx)
    torch.cuda.synchronize()
    first = [{k: v.clone() for k, (v, _) in o.items()} for o in outs]
    for i in (0, 1, 2, 3, 4, 31, 62, 63):
        log("headline frame %d vs oracle" % i)
        spec = gs.edge_spec(synth.recipe_frame(w, h, i, 4), phase=True)
        got = {k: v.cpu().numpy() for k, v in first[i].items()}
        compare(spec, got, spec.run_oracle(), phase_names=("ph",))
    hvx.hvx_batch_autotune(b, stream, 1, ctx=ctx)
    log("tuned: rows %d" % hvx.hvx_batch_query(b, hvx.HVX_QUERY_ROWS_PER_ITEM))
    for persistent in (0, 1):
        hvx.hvx_batch_set_option(b, hvx.HVX_BATCH_PERSISTENT, persistent, ctx=ctx)
        for o in outs:
            for v, _ in o.values():
                v.fill_(0xA5)
        torch.cuda.synchronize()
        log("headline tuned shape, persistent=%d" % persistent)
        hvx.hvx_batch_schedule(b, stream, ctx=ctx)
        torch.cuda.synchronize()
        for i, (a, o) in enumerate(zip(first, outs)):
            for k, (v, _) in o.items():
                assert torch.equal(a[k], v), (i, k, persistent)
    hvx.hvx_release_batch(b)
    for g in graphs:
        hvx.hvx_release_graph(g)


@pytest.mark.parametrize("w,h", [(3840, 2160), (7680, 4320)])
@pytest.mark.parametrize("border", [("replicate", 0), ("constant", 0)])
def test_edge_phase_unfused_fullsize(ctx, w, h, border):
    """Node by node (fusion off: six kernels, every intermediate in device
    memory) at 4K and 8K, REPLICATE and CONSTANT(0), against the oracle."""
    img = synth.edge_image(w, h, seed=w + (border[0] == "constant"))
    spec = gs.edge_spec(img, phase=True, b0=border, b1=border)
    log("unfused edge+phase %dx%d %s" % (w, h, border[0]))
    got, g = run_spec(spec, ctx, fusion=False)
    assert hvx.hvx_graph_query(g, hvx.HVX_QUERY_NUM_KERNELS) == 6
    compare(spec, got, spec.run_oracle(), phase_names=("ph",))
    hvx.hvx_release_graph(g)


def test_edge_phase_8k_batch16(ctx):
    """16 frames of 7680x4320 with the Phase output; CONSTANT(0) Sobel border
    on half of them."""
    w, h, n = 7680, 4320, 16
    specs = [gs.edge_spec(synth.edge_image(w, h, seed=i), phase=True,
                          b1=("constant", 0) if i % 2 else ("replicate", 0)) for i in range(n)]
    graphs, outs, keep = _build_batch(ctx, specs)

    def check(res):
        for i in (0, 15):
            log("8K frame %d vs oracle" % i)
            got = {k: v.cpu().numpy() for k, v in res[i].items()}
            compare(specs[i], got, specs[i].run_oracle(), phase_names=("ph",))

    _run_modes(ctx, graphs, outs, check)
    for g in graphs:
        hvx.hvx_release_graph(g)


def test_mixed_batch_256(ctx):
    """The 256-image mixed batch: W ~ U{320..4096}, H ~ U{240..2160}, kinds
    edge / corner / Gaussian5x5, uniform U8 pixels from seed 1000 + i."""
    shapes = synth.batch_shapes(256, seed=0)
    specs = []
    for (w, h, kind, seed) in shapes:
        img = synth.uniform_u8(w, h, seed)
        if kind == "sobel_edge":
            specs.append(gs.edge_spec(img))
        elif kind == "harris":
            specs.append(gs.corner_spec(img))
        else:
            specs.append(gs.gauss5_spec(img))
    graphs, outs, keep = _build_batch(ctx, specs)
    sample = sorted({0, 255} | set(range(7, 256, 25)))

    def check(res):
        for i in sample:
            w, h, kind, _ = shapes[i]
            log("mixed image %d (%s %dx%d) vs oracle" % (i, kind, w, h))
            got = {k: v.cpu().numpy() for k, v in res[i].items()}
            env = specs[i].run_oracle()
            compare(specs[i], got, env, corner=(kind == "harris"))

    _run_modes(ctx, graphs, outs, check)
    for g in graphs:
        hvx.hvx_release_graph(g)


# ---- F32 operators of the corner graph ---------------------------------------------

def _corner_terms(env, k=0.04):
    sxx, syy, sxy = env["sxx"], env["syy"], env["sxy"]
    return np.abs(sxx * syy) + sxy * sxy + k * (sxx + syy) ** 2


@pytest.mark.parametrize("w,h,b1", [(1920, 1080, ("replicate", 0)), (301, 77, ("constant", 5)),
                                    (64, 9, ("replicate", 0))])
def test_corner_response_f32(ctx, w, h, b1):
    """The response R as a non-virtual F32 output: |R - R64| <= 1e-5 * M with
    M = |Sxx Syy| + Sxy^2 + k (Sxx + Syy)^2, the scale of the terms whose
    cancellation R is."""
    img = synth.corner_image(w, h, seed=w)
    spec = gs.corner_spec(img, b1=b1)
    spec.outputs = {"out": np.uint8, "r": np.float32}
    env = spec.run_oracle()
    log("corner response F32 %dx%d %s" % (w, h, b1))
    got, g = run_spec(spec, ctx)
    r = got["r"].astype(np.float64)
    m = _corner_terms(env)
    err = np.abs(r - env["r"])
    assert np.all(err <= 1e-5 * m), "max excess %g" % (err - 1e-5 * m).max()
    compare(gs.Spec(spec.nodes, spec.inputs, {"out": np.uint8}), {"out": got["out"]}, env, corner=True)


@pytest.mark.parametrize("border", [("replicate", 0), ("constant", 3), ("undefined", 0)])
def test_box5x5_f32_single(ctx, border):
    """Box5x5 over arbitrary F32 values: a 25-term float sum is within
    25 * 2^-24 * sum|x| of the exact sum (the oracle's FP64 sum of |x| gives
    the bound)."""
    w, h = 203, 37
    rng = np.random.default_rng(5)
    x = (rng.standard_normal((h, w)) * 1000).astype(np.float32)
    spec = gs.Spec([gs.N("box5x5_f32", ["in"], ["out"], *border)], {"in": x}, {"out": np.float32})
    env = spec.run_oracle()
    absenv = gs.Spec(spec.nodes, {"in": np.abs(x)}, spec.outputs).run_oracle()
    log("box5x5 f32 %s" % (border,))
    got, _ = run_spec(spec, ctx, fusion=False)
    import oracle
    m = oracle.valid_masks(spec.oracle_graph(), spec.shapes())["out"]
    bound = 25 * 2.0 ** -24 * (absenv["out"] + 25 * abs(border[1]))
    err = np.abs(got["out"].astype(np.float64) - env["out"])
    assert np.all(err[m] <= bound[m])


def test_multiply_f32_exact(ctx):
    """S16 x S16 -> F32 is one correctly rounded product: bit-equal to the
    exact FP64 product rounded to F32."""
    a = synth.uniform_s16(517, 23, seed=1)
    b = synth.uniform_s16(517, 23, seed=2)
    spec = gs.Spec([gs.N("multiply_f32", ["a", "b"], ["out"])], {"a": a, "b": b}, {"out": np.float32})
    env = spec.run_oracle()
    log("multiply f32")
    got, _ = run_spec(spec, ctx, fusion=False)
    assert np.array_equal(got["out"], env["out"].astype(np.float32))


# ---- extremes of the accepted sizes ----------------------------------------------

@pytest.mark.parametrize("w,h", [(65536, 3), (3, 65536), (65535, 2)])
def test_edge_phase_extreme_shapes(ctx, w, h):
    """Widest and tallest images the API accepts (65536), through the fused
    edge+phase kernel and through the node-by-node path."""
    img = synth.edge_image(w, h, seed=w % 97 + h)
    spec = gs.edge_spec(img, phase=True)
    env = spec.run_oracle()
    log("edge extreme %dx%d" % (w, h))
    got, g = run_spec(spec, ctx)
    assert hvx.hvx_graph_query(g, hvx.HVX_QUERY_KERNEL_KIND) == 1
    compare(spec, got, env, phase_names=("ph",))
    unf, _ = run_spec(spec, ctx, fusion=False)
    compare(spec, unf, env, phase_names=("ph",))


def test_empty_and_generic_only_batches(ctx):
    """A batch of no graphs is a no-op; a batch whose graphs all run generated
    kernels has no hand-fused launch: the two graphs, which share their
    generated kernel, run in one launch of it."""
    import torch
    side = torch.cuda.Stream()  # capturable (the null stream is not)
    stream = side.cuda_stream
    b = hvx.hvx_batch_create(ctx, [])
    assert hvx.hvx_batch_query(b, hvx.HVX_QUERY_NUM_OPS) == 0
    hvx.hvx_batch_schedule(b, stream, ctx=ctx)
    torch.cuda.synchronize()
    hvx.hvx_release_batch(b)
    img = synth.edge_image(333, 41, seed=8)
    spec = gs.Spec([gs.N("box3x3", ["in"], ["b"]), gs.N("add", ["in", "b"], ["out"], params={"policy": "wrap"})],
                   {"in": img}, {"out": np.uint8})
    graphs, outs, keep = _build_batch(ctx, [spec, spec])
    b = hvx.hvx_batch_create(ctx, graphs)
    assert hvx.hvx_batch_query(b, hvx.HVX_QUERY_NUM_OPS) == 0
    assert hvx.hvx_batch_query(b, hvx.HVX_QUERY_NUM_KERNELS) == 1
    log("generic-only batch")
    hvx.hvx_batch_schedule(b, stream, ctx=ctx)
    torch.cuda.synchronize()
    env = spec.run_oracle()
    for o in outs:
        compare(spec, {"out": o["out"][0][:, :o["out"][1]].cpu().numpy()}, env)
    hvx.hvx_release_batch(b)
    for g in graphs:
        hvx.hvx_release_graph(g)
