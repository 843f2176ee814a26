"""Host-side tests of the kernels generated per fused group: verification
writes and compiles them (hipRTC needs no device), HVX_OPT_CODEGEN switches
them off, and the groups that the one-operator kernels run with constant
operators are not generated.  No compute call is made."""
import numpy as np
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


def _unsharp(ctx, w=640, h=480):
    g = hvx.hvx_graph_create(ctx)
    a, o = _img(ctx, w, h, k=0), _img(ctx, w, h, k=1)
    v = [hvx.hvx_image_create_virtual(g) for _ in range(3)]
    hvx.hvx_gaussian3x3_node(g, a, v[0])
    hvx.hvx_custom_point_node(g, "a - b", [a, v[0]], hvx.HVX_DF_S16, v[1])
    hvx.hvx_custom_point_node(g, "a * 3 / 2", [v[1]], hvx.HVX_DF_S16, v[2])
    hvx.hvx_custom_point_node(g, "a + b", [a, v[2]], hvx.HVX_DF_U8, o)
    return g


def _q(g, attr):
    return hvx.hvx_graph_query(g, attr)


def test_fused_group_is_generated(ctx):
    g = _unsharp(ctx)
    hvx.hvx_graph_verify(g)
    assert _q(g, hvx.HVX_QUERY_NUM_KERNELS) == 1
    assert _q(g, hvx.HVX_QUERY_NUM_GENERATED) == 1
    hvx.hvx_graph_set_option(g, hvx.HVX_OPT_CODEGEN, 0)
    hvx.hvx_graph_verify(g)
    assert _q(g, hvx.HVX_QUERY_NUM_KERNELS) == 1
    assert _q(g, hvx.HVX_QUERY_NUM_GENERATED) == 0


def test_node_by_node_generates_user_kernels_only(ctx):
    """Node by node: the three user point kernels are generated; the
    Gaussian runs in the one-operator local kernel."""
    g = _unsharp(ctx)
    hvx.hvx_graph_set_option(g, hvx.HVX_OPT_FUSION, 0)
    hvx.hvx_graph_verify(g)
    assert _q(g, hvx.HVX_QUERY_NUM_KERNELS) == 4
    assert _q(g, hvx.HVX_QUERY_NUM_GENERATED) == 3


def test_single_builtin_operators_not_generated(ctx):
    g = hvx.hvx_graph_create(ctx)
    a, b, o = _img(ctx, 100, 50, k=0), _img(ctx, 100, 50, k=1), _img(ctx, 100, 50, k=2)
    hvx.hvx_add_node(g, a, b, hvx.HVX_POLICY_SATURATE, o)
    hvx.hvx_graph_verify(g)
    assert _q(g, hvx.HVX_QUERY_NUM_GENERATED) == 0
    g2 = hvx.hvx_graph_create(ctx)
    hvx.hvx_box3x3_node(g2, a, o)
    hvx.hvx_graph_verify(g2)
    assert _q(g2, hvx.HVX_QUERY_NUM_GENERATED) == 0


def test_same_structure_other_size_and_reduction(ctx):
    """A second image size of the same structure verifies too (the source
    does not depend on the size); a producer fused into a histogram is
    generated with its reduction."""
    for w, h in ((33, 7), (1, 1), (4000, 3)):
        g = _unsharp(ctx, w, h)
        hvx.hvx_graph_verify(g)
        assert _q(g, hvx.HVX_QUERY_NUM_GENERATED) == 1
    g = hvx.hvx_graph_create(ctx)
    a = _img(ctx, 300, 200, k=0)
    buf = hvx.hvx_buffer_from_ptr(ctx, FAKE + (1 << 40), 64 * 4)
    v = hvx.hvx_image_create_virtual(g)
    hvx.hvx_gaussian3x3_node(g, a, v)
    hvx.hvx_histogram_node(g, v, 64, 0, 256, buf)
    hvx.hvx_graph_verify(g)
    assert _q(g, hvx.HVX_QUERY_NUM_KERNELS) == 1
    assert _q(g, hvx.HVX_QUERY_NUM_GENERATED) == 1


def test_generated_window_reads_are_whole_16_byte_lds_reads(ctx, tmp_path, monkeypatch):
    """The LDS window reads of a generated kernel compile to 16-byte reads
    (ds_read_b128), which consecutive lanes spread over consecutive banks.
    Reads narrowed to single dwords at a 16-byte lane stride (ds_read2_b32,
    ds_read_b32) would hit a quarter of the banks.  The source written at
    verification is compiled here with hipcc for gfx950 and its assembly
    inspected."""
    import glob
    import os
    import subprocess
    from paper_2008_11476_amd import build
    monkeypatch.setenv("HVX_GEN_DUMP", str(tmp_path))
    g = hvx.hvx_graph_create(ctx)
    a, o = _img(ctx, 640, 480, k=0), _img(ctx, 640, 480, k=1)
    v = [hvx.hvx_image_create_virtual(g) for _ in range(2)]
    hvx.hvx_gaussian3x3_node(g, a, v[0])
    hvx.hvx_custom_point_node(g, "a - b * 5 / 7", [a, v[0]], hvx.HVX_DF_S16, v[1])  # a source no other test builds
    hvx.hvx_custom_point_node(g, "a + b", [a, v[1]], hvx.HVX_DF_U8, o)
    hvx.hvx_graph_verify(g)
    assert _q(g, hvx.HVX_QUERY_NUM_GENERATED) == 1
    srcs = glob.glob(str(tmp_path / "hvx_gen_*.hip"))
    assert len(srcs) == 1, srcs
    text = open(srcs[0]).read()
    # the hipRTC prelude declares a namespace that the full HIP headers define themselves
    text = text.replace("namespace __hip_internal {}\nusing namespace __hip_internal;\n", "")
    src = tmp_path / "k.hip"
    src.write_text(text)
    csrc = os.path.join(os.path.dirname(build.__file__), "csrc")
    inc = os.path.join(os.path.dirname(os.path.dirname(build.__file__)), "include")
    asm = tmp_path / "k.s"
    r = subprocess.run([build._hipcc(), "-x", "hip", "-O3", "-std=c++17", "--offload-arch=gfx950", "--cuda-device-only",
                        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-S", "-I", csrc, "-I", inc,
                        str(src), "-o", str(asm)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    ops = [ln.split()[0] for ln in asm.read_text().splitlines() if ln.strip().startswith("ds_read")]
    assert ops and all(op == "ds_read_b128" for op in ops), sorted(set(ops))


def test_rank_one_convolve_masks_sum_columns_first(ctx, tmp_path, monkeypatch):
    """A Convolve mask that is the outer product of a column and a row is
    evaluated in interior tiles as column sums shared by a thread's four
    outputs (bit-identical in 32-bit wrapping arithmetic, since the double
    sums agree as integers); other masks, and rank-one masks where it saves
    nothing, keep the direct sum.  Checked on the source written at
    verification."""
    import glob
    import re
    monkeypatch.setenv("HVX_GEN_DUMP", str(tmp_path))
    masks = [(np.outer([1, -2, 0, 3, 1], [2, -1, 5]), 1),       # rank one: 5 rows x 3 columns
             (np.array([[1, 2, 3], [4, 5, 6], [7, 8, 11]]), 1),  # rank three
             (np.outer([3, 0, -3], [6, -12, 6]), 1)]            # rank one, nothing saved
    convs = [hvx.hvx_convolution_create(ctx, m, s) for m, s in masks]
    g = hvx.hvx_graph_create(ctx)
    a, o = _img(ctx, 640, 480, k=0), _img(ctx, 640, 480, k=1)
    v = [hvx.hvx_image_create_virtual(g, 0, 0, hvx.HVX_DF_U8) for _ in range(2)]
    hvx.hvx_convolve_node(g, a, convs[0], v[0])
    hvx.hvx_convolve_node(g, v[0], convs[1], v[1])
    hvx.hvx_convolve_node(g, v[1], convs[2], o)
    hvx.hvx_graph_verify(g)
    assert _q(g, hvx.HVX_QUERY_NUM_GENERATED) == 1
    srcs = glob.glob(str(tmp_path / "hvx_gen_*.hip"))
    assert len(srcs) == 1, srcs
    text = open(srcs[0]).read()
    cols = re.findall(r"const unsigned cs(\d+) = ", text)
    # column sums for the first mask only (in each interior sweep of its
    # stage), window columns x - 1 .. x + 4 of the 3-wide mask
    assert cols and sorted(set(int(c) for c in cols)) == list(range(3, 9)), cols
    assert len(cols) % 6 == 0 and all(cols.count(c) == len(cols) // 6 for c in cols)
    # the column weights (1, -2, 3, 1; the zero dropped) and the row weights
    # (2, -1, 5: 5 through the 24-bit multiplier)
    assert re.search(r"cs3 = 0u \+ \(unsigned\)\(w\[4\]\[3\]\) - 2u \* \(unsigned\)\(w\[3\]\[3\]\) "
                     r"\+ \(unsigned\)__mul24\(\(int\)\(w\[1\]\[3\]\), 3\) \+ \(unsigned\)\(w\[0\]\[3\]\);", text)
    assert "(unsigned)__mul24((int)(cs3), 5)" in text
    for c in convs:
        hvx.hvx_release_convolution(c)
    hvx.hvx_release_graph(g)


def test_outputs_no_later_kernel_reads_use_non_temporal_stores(ctx, tmp_path, monkeypatch):
    """A generated kernel writes a value with non-temporal stores when no
    later kernel of the graph reads it (it would only wait in the caches to
    be written back), and with ordinary stores when a later kernel does.
    Node by node, the three user point kernels of a graph that no other
    test builds each get their own kernel: the two that feed the next one
    store ordinarily, the last one streams."""
    import glob
    import re
    monkeypatch.setenv("HVX_GEN_DUMP", str(tmp_path))
    g = hvx.hvx_graph_create(ctx)
    a, o = _img(ctx, 640, 480, k=0), _img(ctx, 640, 480, k=1)
    v = [hvx.hvx_image_create_virtual(g) for _ in range(2)]
    hvx.hvx_custom_point_node(g, "a * 7 - 3", [a], hvx.HVX_DF_S16, v[0])
    hvx.hvx_custom_point_node(g, "a / 5 + b", [v[0], a], hvx.HVX_DF_S16, v[1])
    hvx.hvx_custom_point_node(g, "a - b * 2", [v[1], a], hvx.HVX_DF_U8, o)
    hvx.hvx_graph_set_option(g, hvx.HVX_OPT_FUSION, 0)
    hvx.hvx_graph_verify(g)
    assert _q(g, hvx.HVX_QUERY_NUM_KERNELS) == 3 and _q(g, hvx.HVX_QUERY_NUM_GENERATED) == 3
    kinds = []
    for src in glob.glob(str(tmp_path / "hvx_gen_*.hip")):
        kinds += re.findall(r"store4<(true|false)>", open(src).read())
    assert sorted(kinds) == ["false", "false", "true"], kinds
    hvx.hvx_release_graph(g)
