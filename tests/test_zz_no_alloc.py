"""GPU test of the allocation-free EqualizeHist entry point: its output must
equal that of hvx_equalize_hist (the same operator with a caller workspace)
and the oracle's, on two calls in a row, the second with a smaller image, so
that stale counts from the first call would show.  Runs alone in a fresh
process as well as after the other tests."""
import numpy as np
import pytest

import oracle.globalops as G
import paper_2008_11476_amd as hvx
import synth
from tests.gpu_util import device_image, log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = hvx.hvx_context_create(0)
    yield c
    hvx.hvx_context_release(c)


def _equalize_both(ctx, img, seed):
    """(output of the workspace form, output of the allocation-free form)."""
    import torch
    h, w = img.shape
    im, keep = device_image(ctx, img, hvx.HVX_DF_U8, seed=seed)
    outs = []
    for k in range(2):
        ob, ov = hvx.alloc_image(h, w, hvx.HVX_DF_U8)
        ov.fill_(0x5A)
        outs.append((hvx.image_from_tensor(ctx, ov, hvx.HVX_DF_U8), ov))
    ws = torch.full((320,), -1, dtype=torch.int32, device="cuda")
    hvx.hvx_equalize_hist(ctx, im, outs[0][0], ws.data_ptr())
    hvx.hvx_equalize_hist_noalloc(ctx, im, outs[1][0])
    torch.cuda.synchronize()
    return outs[0][1].cpu().numpy(), outs[1][1].cpu().numpy(), keep


def test_noalloc_equals_workspace_form_twice(ctx):
    # first a large image with every level present, then a smaller one with
    # a narrow range: counts left over from the first call would change the
    # second mapping
    cases = [(synth.edge_image(1920, 1080, seed=5), 1),
             ((synth.uniform_u8(333, 97, seed=9) // 16 + 60).astype(np.uint8), 2)]
    for img, seed in cases:
        h, w = img.shape
        log("equalize_hist_noalloc %dx%d" % (w, h))
        ref_ws, got, _ = _equalize_both(ctx, img, seed)
        want = G.equalize_hist(img)
        assert np.array_equal(ref_ws, want)
        assert np.array_equal(got, ref_ws)


def test_noalloc_in_place_and_errors(ctx):
    import torch
    img = synth.edge_image(640, 480, seed=3)
    im, keep = device_image(ctx, img, hvx.HVX_DF_U8, seed=4)
    hvx.hvx_equalize_hist_noalloc(ctx, im, im)
    torch.cuda.synchronize()
    assert np.array_equal(keep.cpu().numpy()[:, :640], G.equalize_hist(img))
    ob, ov = hvx.alloc_image(10, 10, hvx.HVX_DF_U8)
    small = hvx.image_from_tensor(ctx, ov, hvx.HVX_DF_U8)
    with pytest.raises(hvx.HvxError):
        hvx.hvx_equalize_hist_noalloc(ctx, im, small)  # size mismatch
