"""GPU parity of the global operators (Table 2: histogram, min/max, mean and
standard deviation) against the oracle: counts, extremes and sums bit-exact,
mean and standard deviation to float rounding."""
import numpy as np
import pytest

import oracle.globalops as G
import paper_2008_11476_amd as hvx
import synth
from tests.gpu_util import device_image, log

pytestmark = pytest.mark.gpu

SIZES = [(1, 1), (15, 3), (17, 2), (67, 45), (1920, 1080), (3840, 2160)]


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = hvx.hvx_context_create(0)
    yield c
    hvx.hvx_context_release(c)


def _img(w, h, seed, kind="edge"):
    if kind == "edge":
        return synth.edge_image(w, h, seed=seed)
    return synth.uniform_u8(w, h, seed=seed)


@pytest.mark.parametrize("w,h", SIZES)
@pytest.mark.parametrize("bins,offset,rng", [(256, 0, 256), (16, 0, 256), (10, 20, 200), (1, 0, 256), (7, 100, 21),
                                             (1, 77, 1), (5, 250, 6), (255, 1, 255)])
def test_histogram(ctx, w, h, bins, offset, rng):
    import torch
    log("histogram %dx%d bins %d offset %d range %d" % (w, h, bins, offset, rng))
    img = _img(w, h, seed=w + bins)
    im, keep = device_image(ctx, img, hvx.HVX_DF_U8, seed=3)
    out = torch.full((bins,), 12345, dtype=torch.int32, device="cuda")  # stale contents are overwritten
    for _ in range(2):  # a second call starts from zero again
        hvx.hvx_histogram(ctx, im, bins, offset, rng, out.data_ptr())
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy().view(np.uint32), G.histogram(img, bins, offset, rng))


def test_histogram_constant_image_all_lanes_collide(ctx):
    import torch
    img = np.full((300, 1000), 200, np.uint8)
    im, keep = device_image(ctx, img, hvx.HVX_DF_U8)
    out = torch.zeros(256, dtype=torch.int32, device="cuda")
    hvx.hvx_histogram(ctx, im, 256, 0, 256, out.data_ptr())
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    assert got[200] == 300 * 1000 and got.sum() == 300 * 1000


@pytest.mark.parametrize("w,h", SIZES)
@pytest.mark.parametrize("dtype", [np.uint8, np.int16])
def test_min_max(ctx, w, h, dtype):
    import torch
    log("min_max %dx%d %s" % (w, h, np.dtype(dtype).name))
    rng = np.random.default_rng(w * h)
    if dtype == np.uint8:
        img = rng.integers(30, 220, (h, w), dtype=np.uint8)
        df = hvx.HVX_DF_U8
    else:
        img = rng.integers(-3000, 3000, (h, w), dtype=np.int16)
        df = hvx.HVX_DF_S16
    # extremes placed in the last column and the last row (ragged tails)
    img[h - 1, w - 1] = np.iinfo(dtype).max if w * h > 1 else img[0, 0]
    img[h // 2, 0] = np.iinfo(dtype).min if w * h > 1 else img[0, 0]
    im, keep = device_image(ctx, img, df, seed=5)
    out = torch.zeros(2, dtype=torch.int32, device="cuda")
    hvx.hvx_min_max(ctx, im, out.data_ptr())
    torch.cuda.synchronize()
    assert tuple(out.cpu().tolist()) == G.min_max(img)


@pytest.mark.parametrize("w,h", SIZES)
@pytest.mark.parametrize("kind", ["edge", "uniform"])
def test_mean_std_dev(ctx, w, h, kind):
    import torch
    log("mean_std_dev %dx%d %s" % (w, h, kind))
    img = _img(w, h, seed=h, kind=kind)
    im, keep = device_image(ctx, img, hvx.HVX_DF_U8, seed=7)
    out = torch.zeros(3, dtype=torch.int64, device="cuda")
    hvx.hvx_mean_std_dev(ctx, im, out.data_ptr())
    torch.cuda.synchronize()
    raw = out.cpu().numpy()
    mean, std, s1, s2 = G.mean_std_dev(img)
    assert int(raw[0]) == s1 and int(raw[1]) == s2
    f = raw[2:3].view(np.float32)
    assert f[0] == np.float32(mean)
    assert abs(float(f[1]) - std) <= 1e-6 * max(std, 1.0)


def test_global_ops_reject_bad_arguments(ctx):
    import torch
    img = synth.uniform_u8(64, 4, seed=1)
    im, keep = device_image(ctx, img, hvx.HVX_DF_U8)
    s16, keep2 = device_image(ctx, img.astype(np.int16), hvx.HVX_DF_S16)
    buf = torch.zeros(512, dtype=torch.int32, device="cuda")
    for bins, off, rng in ((0, 0, 256), (257, 0, 256), (10, 0, 5), (4, 200, 100)):
        with pytest.raises(hvx.HvxError):
            hvx.hvx_histogram(ctx, im, bins, off, rng, buf.data_ptr())
    with pytest.raises(hvx.HvxError):
        hvx.hvx_histogram(ctx, s16, 16, 0, 256, buf.data_ptr())
    with pytest.raises(hvx.HvxError):
        hvx.hvx_mean_std_dev(ctx, s16, buf.data_ptr())
    with pytest.raises(hvx.HvxError):
        hvx.hvx_mean_std_dev(ctx, im, buf.data_ptr() + 4)
    with pytest.raises(hvx.HvxError):
        hvx.hvx_min_max(ctx, im, None)


@pytest.mark.parametrize("w,h", SIZES)
@pytest.mark.parametrize("dtype", [np.uint8, np.int16])
def test_min_max_count(ctx, w, h, dtype):
    """The MinMaxLoc counts: narrow values so that both extremes repeat,
    and a constant image where they coincide."""
    import torch
    log("min_max_count %dx%d %s" % (w, h, np.dtype(dtype).name))
    rng = np.random.default_rng(w + h)
    df = hvx.HVX_DF_U8 if dtype == np.uint8 else hvx.HVX_DF_S16
    for img in (rng.integers(-2 if dtype == np.int16 else 7, 12, (h, w)).astype(dtype),
                np.full((h, w), 5, dtype)):
        im, keep = device_image(ctx, img, df, seed=9)
        out = torch.full((1032,), 77, dtype=torch.int32, device="cuda")  # 4128 bytes
        hvx.hvx_min_max_count(ctx, im, out.data_ptr())
        torch.cuda.synchronize()
        assert tuple(out.cpu().tolist()[:4]) == G.min_max_count(img)


@pytest.mark.parametrize("w,h", SIZES)
@pytest.mark.parametrize("kind", ["edge", "uniform", "narrow", "constant"])
def test_equalize_hist(ctx, w, h, kind):
    import torch
    log("equalize_hist %dx%d %s" % (w, h, kind))
    if kind == "narrow":
        img = (synth.uniform_u8(w, h, seed=w) // 32 + 100).astype(np.uint8)
    elif kind == "constant":
        img = np.full((h, w), 77, np.uint8)
    else:
        img = _img(w, h, seed=h + 1, kind=kind)
    want = G.equalize_hist(img)
    im, keep = device_image(ctx, img, hvx.HVX_DF_U8, seed=11)
    ob, ov = hvx.alloc_image(h, w, hvx.HVX_DF_U8)
    om = hvx.image_from_tensor(ctx, ov, hvx.HVX_DF_U8)
    ws = torch.full((320,), -1, dtype=torch.int32, device="cuda")
    hvx.hvx_equalize_hist(ctx, im, om, ws.data_ptr())
    hvx.hvx_equalize_hist(ctx, im, im, ws.data_ptr())  # in place
    torch.cuda.synchronize()
    assert np.array_equal(ov.cpu().numpy(), want)
    got_in_place = keep.cpu().numpy()[:, :w]
    assert np.array_equal(got_in_place, want)
    with pytest.raises(hvx.HvxError):
        hvx.hvx_equalize_hist(ctx, im, om, ws.data_ptr() + 2)


@pytest.mark.parametrize("w,h", SIZES)
@pytest.mark.parametrize("dtype", [np.uint8, np.int16])
def test_min_max_loc(ctx, w, h, dtype):
    """Locations compared as sets when they fit; when an extreme occurs more
    often than the capacity, every kept location must hold the extreme and
    be distinct.  Counts are always the full counts."""
    import torch
    log("min_max_loc %dx%d %s" % (w, h, np.dtype(dtype).name))
    rng = np.random.default_rng(3 * w + h)
    df = hvx.HVX_DF_U8 if dtype == np.uint8 else hvx.HVX_DF_S16
    for img in (rng.integers(0, 200, (h, w)).astype(dtype), rng.integers(-1 if dtype == np.int16 else 4, 9,
                                                                          (h, w)).astype(dtype)):
        mn, mx, cmin, cmax, lmin, lmax = G.min_max_loc(img)
        cap = min(w * h, 5000)
        im, keep = device_image(ctx, img, df, seed=13)
        res = torch.full((1032,), 99, dtype=torch.int32, device="cuda")  # 4128 bytes
        lmn = torch.full((2 * cap,), -1, dtype=torch.int32, device="cuda")
        lmx = torch.full((2 * cap,), -1, dtype=torch.int32, device="cuda")
        hvx.hvx_min_max_loc(ctx, im, res.data_ptr(), lmn.data_ptr(), lmx.data_ptr(), cap)
        torch.cuda.synchronize()
        assert tuple(res.cpu().tolist()[:4]) == (mn, mx, cmin, cmax)
        for got, want, val, cnt in ((lmn, lmin, mn, cmin), (lmx, lmax, mx, cmax)):
            pts = [tuple(p) for p in got.cpu().numpy().reshape(-1, 2)[:min(cnt, cap)].tolist()]
            if cnt <= cap:
                assert sorted(pts) == sorted(want)
            else:
                assert len(set(pts)) == cap
                assert all(0 <= x < w and 0 <= y < h and img[y, x] == val for x, y in pts)


def test_global_ops_replay_from_a_hip_graph(ctx):
    """The calls capture into a HIP graph (their result buffers are set by a
    kernel, not a memset); each replay, after eager changes to the input,
    matches the oracle on the input as it then is."""
    import torch
    w, h = 300, 70
    img = synth.uniform_u8(w, h, seed=21)
    im, dev = device_image(ctx, img, hvx.HVX_DF_U8, seed=1)
    hist = torch.zeros(256, dtype=torch.int32, device="cuda")
    mm = torch.zeros(2, dtype=torch.int32, device="cuda")
    ms = torch.zeros(3, dtype=torch.int64, device="cuda")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(side):
        with torch.cuda.graph(graph, stream=side):
            s = torch.cuda.current_stream().cuda_stream
            hvx.hvx_histogram(ctx, im, 256, 0, 256, hist.data_ptr(), s)
            hvx.hvx_min_max(ctx, im, mm.data_ptr(), s)
            hvx.hvx_mean_std_dev(ctx, im, ms.data_ptr(), s)
    torch.cuda.current_stream().wait_stream(side)
    for rep in range(3):
        cur = (img.astype(np.int32) * (rep + 1) // 3).astype(np.uint8)
        dev[:, :w].copy_(torch.from_numpy(cur))  # eager work between replays
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        log("graph replay %d" % rep)
        assert np.array_equal(hist.cpu().numpy().view(np.uint32), G.histogram(cur, 256, 0, 256))
        assert tuple(mm.cpu().tolist()) == G.min_max(cur)
        mean, std, s1, s2 = G.mean_std_dev(cur)
        raw = ms.cpu().numpy()
        assert int(raw[0]) == s1 and int(raw[1]) == s2
