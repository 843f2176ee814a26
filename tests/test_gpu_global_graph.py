"""GPU parity of global operators as graph nodes (Table 2) against the
node-by-node oracle: each operator alone (the streaming reduction kernels),
fused with the point and local operators that produce its input (the tile
kernel reduces the producer's values without writing them to memory), next
to image outputs of the same kernel, two per kernel, with the locations of
MinMaxLoc and EqualizeHist in later phases, and node by node.  Counts,
extremes, sums and images bit-exact; mean and standard deviation to float
rounding; location lists checked as sets (truncated lists for validity)."""
import numpy as np
import pytest

import paper_2008_11476_amd as hvx
import synth
from tests import graphspec as gs
from tests.gpu_util import log, run_spec

pytestmark = pytest.mark.gpu

SIZES = [(1, 1), (67, 45), (641, 479), (1920, 1080)]
N = gs.N


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = hvx.hvx_context_create(0)
    yield c
    hvx.hvx_context_release(c)


def _check_buffers(spec, got, env):
    """Compare every result buffer of `spec` with the oracle's value."""
    for node in spec.nodes:
        if node.op == "histogram":
            name = node.outs[0]
            bins = node.params["bins"]
            assert np.array_equal(got[name].view(np.uint32)[:bins], env[name]), name
        elif node.op == "min_max":
            name = node.outs[0]
            assert tuple(got[name].view(np.int32)[:2].tolist()) == env[name], name
        elif node.op == "min_max_loc":
            name = node.outs[0]
            r = got[name].view(np.int32)
            mn, mx, cmin, cmax = env[name]
            assert tuple(r[:4].tolist()) == (mn, mx, cmin, cmax), (name, r[:4], env[name])
            cap = node.params.get("capacity", 0)
            if cap:
                lname = node.outs[1]
                src = env[node.ins[0]]
                lmin, lmax = env[lname]
                locs = got[lname].view(np.uint32)
                assert r[4] == min(cmin, cap) and r[5] == min(cmax, cap), (r[4:6], cmin, cmax, cap)
                for k, (want, val, count) in enumerate(((lmin, mn, cmin), (lmax, mx, cmax))):
                    pairs = locs[2 * cap * k: 2 * cap * k + 2 * min(count, cap)].reshape(-1, 2)
                    seen = set(map(tuple, pairs.tolist()))
                    assert len(seen) == len(pairs), "duplicate locations"
                    if count <= cap:
                        assert seen == set(want), "location set differs"
                    else:  # a truncated list: every entry a pixel of that value
                        xs, ys = pairs[:, 0], pairs[:, 1]
                        assert (xs < src.shape[1]).all() and (ys < src.shape[0]).all()
                        assert (src[ys, xs] == val).all()
        elif node.op == "mean_std_dev":
            name = node.outs[0]
            mean, std, s1, s2 = env[name]
            assert tuple(got[name].view(np.uint64)[:2].tolist()) == (s1, s2), name
            f = got[name].view(np.float32)[4:6]
            assert abs(f[0] - mean) <= 1e-6 * max(1.0, abs(mean)) and abs(f[1] - std) <= 1e-5 * max(1.0, std)


def _run(ctx, spec, **kw):
    env = spec.run_oracle()
    got, g = run_spec(spec, ctx, **kw)
    for name in spec.outputs:
        assert np.array_equal(got[name], env[name]), name
    _check_buffers(spec, got, env)
    return g


def _img(w, h, seed, kind="edge"):
    return synth.edge_image(w, h, seed=seed) if kind == "edge" else synth.uniform_u8(w, h, seed=seed)


@pytest.mark.parametrize("w,h", SIZES)
def test_global_nodes_alone(ctx, w, h):
    log("global nodes alone %dx%d" % (w, h))
    img = _img(w, h, seed=w)
    specs = [
        gs.Spec([N("histogram", ["in"], ["hist"], params={"bins": 256})], {"in": img}, {}, buffers={"hist": 1024}),
        gs.Spec([N("histogram", ["in"], ["hist"], params={"bins": 7, "offset": 100, "range": 21})], {"in": img}, {},
                buffers={"hist": 64}),
        gs.Spec([N("min_max", ["in"], ["mm"])], {"in": img}, {}, buffers={"mm": 8}),
        gs.Spec([N("min_max_loc", ["in"], ["mm", "locs"], params={"capacity": 32})], {"in": img}, {},
                buffers={"mm": 4128, "locs": 16 * 32}),
        gs.Spec([N("mean_std_dev", ["in"], ["ms"])], {"in": img}, {}, buffers={"ms": 24}),
        gs.Spec([N("equalize_hist", ["in"], ["out"])], {"in": img}, {"out": np.uint8}),
    ]
    for spec in specs:
        g = _run(ctx, spec)
        assert hvx.hvx_graph_query(g, hvx.HVX_QUERY_KERNEL_KIND) == 4


@pytest.mark.parametrize("w,h", [(67, 45), (641, 479)])
def test_min_max_loc_s16_alone_and_rare_extremes(ctx, w, h):
    rng = np.random.default_rng(w)
    img = rng.integers(-3000, 3000, (h, w), dtype=np.int16)
    img[h - 1, w - 1] = 32767
    img[h // 2, 0] = -32768
    img[0, w // 3] = -32768
    spec = gs.Spec([N("min_max_loc", ["in"], ["mm", "locs"], params={"capacity": 4})], {"in": img}, {},
                   buffers={"mm": 4128, "locs": 16 * 4})
    _run(ctx, spec)


@pytest.mark.parametrize("w,h", SIZES)
@pytest.mark.parametrize("border", [("replicate", 0), ("constant", 0), ("constant", 200)])
def test_producer_fused_into_reduction(ctx, w, h, border):
    log("fused reductions %dx%d %s" % (w, h, border))
    img = _img(w, h, seed=w + 7)
    # Gaussian3x3 -> histogram, nothing materialised, one kernel
    spec = gs.Spec([N("gaussian3x3", ["in"], ["g"], *border), N("histogram", ["g"], ["hist"], params={"bins": 256})],
                   {"in": img}, {}, buffers={"hist": 1024})
    g = _run(ctx, spec)
    assert hvx.hvx_graph_query(g, hvx.HVX_QUERY_NUM_KERNELS) == 1
    assert hvx.hvx_graph_query(g, hvx.HVX_QUERY_SCRATCH_BYTES) == 0
    # Gaussian5x5 -> mean and standard deviation
    spec = gs.Spec([N("gaussian5x5", ["in"], ["g"], *border), N("mean_std_dev", ["g"], ["ms"])],
                   {"in": img}, {}, buffers={"ms": 24})
    _run(ctx, spec)
    # Sobel -> Magnitude (S16) -> MinMaxLoc counts; median -> min/max
    spec = gs.Spec([N("sobel3x3", ["in"], ["gx", "gy"], *border), N("magnitude", ["gx", "gy"], ["m"]),
                    N("min_max_loc", ["m"], ["mm"])], {"in": img}, {}, buffers={"mm": 4128})
    _run(ctx, spec)
    spec = gs.Spec([N("median3x3", ["in"], ["md"], *border), N("min_max", ["md"], ["mm"])],
                   {"in": img}, {}, buffers={"mm": 8})
    _run(ctx, spec)


@pytest.mark.parametrize("w,h", SIZES)
def test_image_outputs_and_two_reductions_in_one_kernel(ctx, w, h):
    img = _img(w, h, seed=w + 11, kind="uniform")
    spec = gs.Spec([N("gaussian3x3", ["in"], ["out"]), N("threshold", ["out"], ["t"], params={"thresh": 120}),
                    N("histogram", ["t"], ["hist"], params={"bins": 2}), N("min_max_loc", ["out"], ["mm"])],
                   {"in": img}, {"out": np.uint8}, buffers={"hist": 8, "mm": 4128})
    g = _run(ctx, spec)
    assert hvx.hvx_graph_query(g, hvx.HVX_QUERY_NUM_KERNELS) == 1
    # three reductions: split node by node, same results
    spec = gs.Spec([N("gaussian3x3", ["in"], ["g"]), N("min_max", ["g"], ["a"]), N("mean_std_dev", ["g"], ["b"]),
                    N("histogram", ["g"], ["c"], params={"bins": 16})], {"in": img}, {},
                   buffers={"a": 8, "b": 24, "c": 64})
    g = _run(ctx, spec)
    assert hvx.hvx_graph_query(g, hvx.HVX_QUERY_NUM_KERNELS) == 4


@pytest.mark.parametrize("w,h", SIZES)
@pytest.mark.parametrize("fusion", [True, False])
def test_later_phases(ctx, w, h, fusion):
    log("phases %dx%d fusion %s" % (w, h, fusion))
    img = _img(w, h, seed=w + 3)
    # EqualizeHist -> Gaussian3x3: mapping first, then mapping and Gaussian fused
    spec = gs.Spec([N("equalize_hist", ["in"], ["e"]), N("gaussian3x3", ["e"], ["out"])], {"in": img},
                   {"out": np.uint8})
    _run(ctx, spec, fusion=fusion)
    # Gaussian3x3 -> EqualizeHist: Gaussian fused into the histogram, kept for the mapping
    spec = gs.Spec([N("gaussian3x3", ["in"], ["g"]), N("equalize_hist", ["g"], ["out"])], {"in": img},
                   {"out": np.uint8})
    _run(ctx, spec, fusion=fusion)
    # MinMaxLoc of a Gaussian5x5 with locations (second pass over the kept Gaussian)
    for cap in (3, 100000):
        spec = gs.Spec([N("gaussian5x5", ["in"], ["g"]), N("min_max_loc", ["g"], ["mm", "locs"],
                                                            params={"capacity": cap})],
                       {"in": img}, {}, buffers={"mm": 4128, "locs": 16 * cap})
        _run(ctx, spec, fusion=fusion)


def test_repeated_process_calls_start_clean(ctx):
    import torch
    img = _img(640, 480, seed=5)
    spec = gs.Spec([N("gaussian3x3", ["in"], ["g"]), N("histogram", ["g"], ["hist"], params={"bins": 256}),
                    N("min_max_loc", ["g"], ["mm"]), ], {"in": img}, {}, buffers={"hist": 1024, "mm": 4128})
    env = spec.run_oracle()
    held = {}
    got, g = run_spec(spec, ctx, keep=held)
    _check_buffers(spec, got, env)
    for _ in range(3):  # results are reset by each call
        hvx.hvx_graph_process(g, ctx=ctx)
    torch.cuda.synchronize()
    again = {name: t.cpu().numpy() for name, t in held["buffers"].items()}
    _check_buffers(spec, again, env)
