"""One graph description, built twice: as an hvx graph (through the C ABI)
and as an oracle graph.  Test infrastructure only."""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

import oracle
import paper_2008_11476_amd as hvx

BORDER = {"undefined": hvx.HVX_BORDER_UNDEFINED, "constant": hvx.HVX_BORDER_CONSTANT,
          "replicate": hvx.HVX_BORDER_REPLICATE, "mirror": hvx.HVX_BORDER_MIRROR,
          "repeat": hvx.HVX_BORDER_REPEAT}
DF_OF_DTYPE = {np.dtype(np.uint8): hvx.HVX_DF_U8, np.dtype(np.int16): hvx.HVX_DF_S16,
               np.dtype(np.float32): hvx.HVX_DF_F32, np.dtype(np.float64): hvx.HVX_DF_F32}


@dataclass
class N:
    op: str
    ins: list
    outs: list
    border: str = "replicate"
    c: int = 0
    params: dict = field(default_factory=dict)


@dataclass
class Spec:
    nodes: list
    inputs: dict    # name -> numpy array (UYVY: (H, 2W) uint8 with params["uyvy"])
    outputs: dict   # name -> numpy dtype of a non-virtual output
    uyvy: tuple = ()  # input names holding UYVY frames
    buffers: dict = field(default_factory=dict)  # name -> bytes of a global operator's result buffer

    def oracle_graph(self):
        g = oracle.Graph()
        for n in self.nodes:
            g.add(n.op, n.ins, n.outs, border=n.border, constant=n.c, **n.params)
        return g

    def run_oracle(self):
        return oracle.run(self.oracle_graph(), dict(self.inputs))

    def shapes(self):
        out = {}
        for k, v in self.inputs.items():
            out[k] = (v.shape[0], v.shape[1] // 2) if k in self.uyvy else v.shape[:2]
        return out


def build_hvx(spec: Spec, ctx, images: dict):
    """Create the hvx graph.  ``images`` maps every non-virtual name to an hvx
    image handle; other names become virtual images of the graph."""
    g = hvx.hvx_graph_create(ctx)
    virt = {}

    def im(name):
        if name is None:
            return None
        if name in images:
            return images[name]
        if name not in virt:
            virt[name] = hvx.hvx_image_create_virtual(g, ctx=ctx)
        return virt[name]

    nodes = []
    for n in spec.nodes:
        a = [im(x) for x in n.ins]
        o = [im(x) for x in n.outs]
        p = n.params
        if n.op == "channel_extract_y":
            h = hvx.hvx_channel_extract_node(g, a[0], hvx.HVX_CHANNEL_Y, o[0], ctx=ctx)
        elif n.op == "gaussian3x3":
            h = hvx.hvx_gaussian3x3_node(g, a[0], o[0], ctx=ctx)
        elif n.op == "gaussian5x5":
            h = hvx.hvx_gaussian5x5_node(g, a[0], o[0], ctx=ctx)
        elif n.op == "box3x3":
            h = hvx.hvx_box3x3_node(g, a[0], o[0], ctx=ctx)
        elif n.op in ("dilate3x3", "erode3x3", "median3x3"):
            h = getattr(hvx, "hvx_%s_node" % n.op)(g, a[0], o[0], ctx=ctx)
        elif n.op == "nonlinear":
            fn = {"median": hvx.HVX_NONLINEAR_MEDIAN, "min": hvx.HVX_NONLINEAR_MIN, "max": hvx.HVX_NONLINEAR_MAX}
            h = hvx.hvx_nonlinear_filter_node(g, fn[p["func"]], a[0], p["mask"], o[0], ctx=ctx)
        elif n.op == "custom_point":
            h = hvx.hvx_custom_point_node(g, p["expr"], a, DF_OF_DTYPE[np.dtype(p["out_dtype"])], o[0], ctx=ctx)
        elif n.op == "custom_local":
            h = hvx.hvx_custom_local_node(g, p["expr"], a[0], DF_OF_DTYPE[np.dtype(p["out_dtype"])], o[0], ctx=ctx)
        elif n.op == "nonmax":
            h = hvx.hvx_non_max_suppression_node(g, a[0], p.get("win", 3), o[0], ctx=ctx)
        elif n.op == "box5x5_f32":
            h = hvx.hvx_box5x5_f32_node(g, a[0], o[0], ctx=ctx)
        elif n.op == "sobel3x3":
            h = hvx.hvx_sobel3x3_node(g, a[0], o[0], o[1] if len(o) > 1 else None, ctx=ctx)
        elif n.op == "magnitude":
            h = hvx.hvx_magnitude_node(g, a[0], a[1], o[0], ctx=ctx)
        elif n.op == "phase":
            h = hvx.hvx_phase_node(g, a[0], a[1], o[0], ctx=ctx)
        elif n.op == "add":
            pol = hvx.HVX_POLICY_SATURATE if p.get("policy", "saturate") == "saturate" else hvx.HVX_POLICY_WRAP
            h = hvx.hvx_add_node(g, a[0], a[1], pol, o[0], ctx=ctx)
        elif n.op == "multiply_f32":
            h = hvx.hvx_multiply_f32_node(g, a[0], a[1], o[0], ctx=ctx)
        elif n.op == "harris_response":
            h = hvx.hvx_harris_response_node(g, a[0], a[1], a[2], p.get("k", 0.04), o[0], ctx=ctx)
        elif n.op == "threshold":
            h = hvx.hvx_threshold_node(g, a[0], p["thresh"], p.get("true_v", 255), p.get("false_v", 0), o[0],
                                       ctx=ctx)
        elif n.op == "convolve":
            conv = hvx.hvx_convolution_create(ctx, p["coeffs"], p["scale"])
            h = hvx.hvx_convolve_node(g, a[0], conv, o[0], ctx=ctx)
        elif n.op == "histogram":
            h = hvx.hvx_histogram_node(g, a[0], p["bins"], p.get("offset", 0), p.get("range", 256), o[0], ctx=ctx)
        elif n.op == "min_max":
            h = hvx.hvx_min_max_node(g, a[0], o[0], ctx=ctx)
        elif n.op == "min_max_loc":
            h = hvx.hvx_min_max_loc_node(g, a[0], o[0], o[1] if len(o) > 1 else None, p.get("capacity", 0),
                                         ctx=ctx)
        elif n.op == "mean_std_dev":
            h = hvx.hvx_mean_std_dev_node(g, a[0], o[0], ctx=ctx)
        elif n.op == "equalize_hist":
            h = hvx.hvx_equalize_hist_node(g, a[0], o[0], ctx=ctx)
        else:
            raise ValueError(n.op)
        if n.border != "replicate" or n.c:
            hvx.hvx_node_set_border(h, BORDER[n.border], n.c, ctx=ctx)
        nodes.append(h)
    return g, nodes, virt


# ---- the graphs of the workloads -------------------------------------------------

def edge_spec(img, phase=False, b0=("replicate", 0), b1=("replicate", 0), thresh=100):
    nodes = [N("gaussian3x3", ["in"], ["g"], *b0),
             N("sobel3x3", ["g"], ["gx", "gy"], *b1),
             N("magnitude", ["gx", "gy"], ["mag"]),
             N("threshold", ["mag"], ["out"], params={"thresh": thresh})]
    outs = {"out": np.uint8}
    if phase:
        nodes.append(N("phase", ["gx", "gy"], ["ph"]))
        outs["ph"] = np.uint8
    return Spec(nodes, {"in": img}, outs)


def corner_spec(img, b0=("replicate", 0), b1=("replicate", 0), k=0.04, thresh=1e6):
    nodes = [N("sobel3x3", ["in"], ["gx", "gy"], *b0),
             N("multiply_f32", ["gx", "gx"], ["pxx"]),
             N("multiply_f32", ["gy", "gy"], ["pyy"]),
             N("multiply_f32", ["gx", "gy"], ["pxy"]),
             N("box5x5_f32", ["pxx"], ["sxx"], *b1),
             N("box5x5_f32", ["pyy"], ["syy"], *b1),
             N("box5x5_f32", ["pxy"], ["sxy"], *b1),
             N("harris_response", ["sxx", "syy", "sxy"], ["r"], params={"k": k}),
             N("threshold", ["r"], ["out"], params={"thresh": thresh})]
    return Spec(nodes, {"in": img}, {"out": np.uint8})


def gauss5_spec(img, b=("replicate", 0)):
    return Spec([N("gaussian5x5", ["in"], ["out"], *b)], {"in": img}, {"out": np.uint8})


def uyvy_gauss5_spec(frame, b=("replicate", 0)):
    return Spec([N("channel_extract_y", ["in"], ["y"]), N("gaussian5x5", ["y"], ["out"], *b)],
                {"in": frame}, {"out": np.uint8}, uyvy=("in",))


def listing1_spec(frame, thresh=100):
    """The edge-detection example of Section 3.1 (Magnitude fed gy twice)."""
    return Spec([N("channel_extract_y", ["in"], ["v0"]),
                 N("gaussian3x3", ["v0"], ["v1"]),
                 N("sobel3x3", ["v1"], ["v2", "v3"]),
                 N("magnitude", ["v3", "v3"], ["v4"]),
                 N("threshold", ["v4"], ["out"], params={"thresh": thresh})],
                {"in": frame}, {"out": np.uint8}, uyvy=("in",))
