"""The autotuner's plan choices (Section 6.3: whether fusing pays off is
measured, not assumed): it times the fused plan, plans cut at values inside
the fused group and the tiles of the generated kernels, keeps the fastest in
the tune cache, and every plan gives the same outputs bit for bit.  Plans
written into a cache file apply to any graph built the same way."""
import json

import numpy as np
import pytest

import paper_2008_11476_amd as hvx
import synth
from tests.gpu_util import compare, log, run_spec
from tests.test_gpu_custom import unsharp_spec

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = hvx.hvx_context_create(0)
    yield c
    hvx.hvx_context_release(c)


def _read(keep):
    import torch
    torch.cuda.synchronize()
    out = {}
    for name, (t, w, dt) in keep["outputs"].items():
        a = t.cpu().numpy()
        out[name] = (a.view(dt) if a.dtype != dt else a)[:, :w]
    return out


def _plan_entry(path):
    d = json.loads(open(path).read())
    keys = [k for k in d if k.startswith("plan|")]
    assert len(keys) == 1, keys
    return keys[0], d[keys[0]]


def test_autotune_records_a_plan_with_identical_outputs(ctx, tmp_path):
    import torch
    img = synth.edge_image(1920, 1080, seed=3)
    spec = unsharp_spec(img)
    env = spec.run_oracle()
    keep = {}
    log("tune plan: default")
    got, g = run_spec(spec, ctx, keep=keep)
    compare(spec, got, env)
    log("tune plan: autotune")
    hvx.hvx_graph_autotune(g, torch.cuda.current_stream().cuda_stream, 3, ctx=ctx)
    hvx.hvx_graph_process(g, ctx=ctx)
    tuned = _read(keep)
    assert np.array_equal(tuned["out"], got["out"])
    path = tmp_path / "tune.json"
    hvx.hvx_context_save_tune_cache(ctx, str(path))
    key, entry = _plan_entry(path)
    assert len(entry) == 5 and isinstance(entry[3], list) and isinstance(entry[4], list)
    assert entry[2] > 0  # microseconds of the chosen plan


@pytest.mark.parametrize("w,h", [(1920, 1080), (131, 29)])
def test_cached_plan_choices_differ_from_the_default_with_identical_outputs(ctx, tmp_path, w, h):
    """A tuned plan differs from the default one (fusion cut at every value,
    i.e. node by node; or another tile for the generated kernel) and gives
    the same outputs, bit for bit, as the default plan and the oracle."""
    import torch
    img = synth.edge_image(w, h, seed=w)
    spec = unsharp_spec(img)
    env = spec.run_oracle()
    base, g0 = run_spec(spec, ctx)
    assert hvx.hvx_graph_query(g0, hvx.HVX_QUERY_NUM_KERNELS) == 1
    default_tile = hvx.hvx_graph_query(g0, hvx.HVX_QUERY_GEN_TILE)
    assert default_tile != 0
    # the key of this graph's plan choices, from a tuned copy in its own context
    c1 = hvx.hvx_context_create(0)
    try:
        keep = {}
        _, g1 = run_spec(spec, c1, keep=keep)
        hvx.hvx_graph_autotune(g1, torch.cuda.current_stream().cuda_stream, 1, ctx=c1)
        path = tmp_path / "tune.json"
        hvx.hvx_context_save_tune_cache(c1, str(path))
    finally:
        hvx.hvx_context_release(c1)
    key, _ = _plan_entry(path)
    other = (32 << 16 | 16) if default_tile != (32 << 16 | 16) else (64 << 16 | 32)
    for entry, check in (([0, 1, 1.0, list(range(64)), []], "cuts"),
                         ([0, 1, 1.0, [], [[0, other >> 16, other & 0xFFFF]]], "tile")):
        forced = tmp_path / ("forced_%s.json" % check)
        forced.write_text(json.dumps({key: entry}))
        c2 = hvx.hvx_context_create(0)
        try:
            hvx.hvx_context_load_tune_cache(c2, str(forced))
            log("tune plan: forced %s %dx%d" % (check, w, h))
            got, g2 = run_spec(spec, c2)
            if check == "cuts":
                assert hvx.hvx_graph_query(g2, hvx.HVX_QUERY_NUM_KERNELS) == 4
                assert hvx.hvx_graph_query(g2, hvx.HVX_QUERY_PLAN_CUTS) > 0
            else:
                assert hvx.hvx_graph_query(g2, hvx.HVX_QUERY_NUM_KERNELS) == 1
                assert hvx.hvx_graph_query(g2, hvx.HVX_QUERY_GEN_TILE) == other
            assert np.array_equal(got["out"], base["out"])
            compare(spec, got, env)
        finally:
            hvx.hvx_context_release(c2)


def test_plan_cut_inside_a_diamond_keeps_dependency_order(ctx):
    """Cutting one value of a fused group whose operators also meet through
    another path: the groups launch after the groups they read."""
    import torch
    img = synth.edge_image(300, 77, seed=9)
    from tests import graphspec as gs
    spec = gs.Spec([gs.N("gaussian3x3", ["in"], ["g"]),
                    gs.N("box3x3", ["in"], ["b"]),
                    gs.N("custom_point", ["g", "b"], ["d"], params={"expr": "a - b", "out_dtype": np.int16}),
                    gs.N("custom_point", ["d", "g"], ["out"], params={"expr": "a + b", "out_dtype": np.uint8})],
                   {"in": img}, {"out": np.uint8})
    env = spec.run_oracle()
    base, g0 = run_spec(spec, ctx)
    compare(spec, base, env)
    keep = {}
    _, g1 = run_spec(spec, ctx, keep=keep)
    hvx.hvx_graph_autotune(g1, torch.cuda.current_stream().cuda_stream, 1, ctx=ctx)
    hvx.hvx_graph_process(g1, ctx=ctx)
    assert np.array_equal(_read(keep)["out"], base["out"])


def test_autotune_graph_with_global_operators(ctx):
    """Plans of a producer fused into global operators (and the plan that
    cuts it off) agree on every result word the operators define; the
    reductions' workspace words may differ between launch shapes."""
    import torch
    from tests import graphspec as gs
    from tests.test_gpu_global_graph import _check_buffers
    img = synth.edge_image(1280, 720, seed=2)
    spec = gs.Spec([gs.N("gaussian5x5", ["in"], ["g"]),
                    gs.N("histogram", ["g"], ["hist"], params={"bins": 64, "offset": 0, "range": 256}),
                    gs.N("min_max_loc", ["g"], ["mm", "locs"], params={"capacity": 32}),
                    gs.N("mean_std_dev", ["g"], ["ms"])],
                   {"in": img}, {}, buffers={"hist": 8192, "mm": 4128, "locs": 2 * 32 * 8, "ms": 64})
    env = spec.run_oracle()
    keep = {}
    got, g = run_spec(spec, ctx, keep=keep)
    _check_buffers(spec, got, env)
    log("tune plan: global operators")
    hvx.hvx_graph_autotune(g, torch.cuda.current_stream().cuda_stream, 2, ctx=ctx)
    hvx.hvx_graph_process(g, ctx=ctx)
    torch.cuda.synchronize()
    tuned = {name: t.cpu().numpy() for name, t in keep["buffers"].items()}
    _check_buffers(spec, tuned, env)
