"""CPU reference (oracle) for OpenVX-style image graphs.

TEST INFRASTRUCTURE ONLY: only the tests, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code
with the GPU library and never imports it.

The oracle is a plain node-by-node executor (Section 3.1): nodes run one at a
time in dependency order, every intermediate image is materialised at full
size in its own element type, and each node applies its own border mode to
its own inputs.  Dead-computation elimination, transfer reduction and fusion
(Sections 5.2.1, 5.2.2, 6.3) are optimisations that must reach exactly this
result, so the plain execution is the reference for all of them.

Global operators (Table 2: histogram, min/max, MinMaxLoc, mean and
standard deviation, EqualizeHist) are nodes like the others: they run in
the same order over the materialised image they read, with the arithmetic
of ``globalops.py``, and their results are kept under their output names.

The per-node arithmetic lives in ``hvx_oracle.c`` (plain C, compiled with gcc
on first use).  Real-valued nodes (the corner graph) run in double precision:
their images are ``float64`` arrays here.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hvx_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

BORDERS = {"undefined": 0, "constant": 1, "replicate": 2, "mirror": 3, "repeat": 4}

# Window radius of each local operator (point operators have radius 0).
RADIUS = {"gaussian3x3": 1, "gaussian5x5": 2, "box3x3": 1, "sobel3x3": 1, "box5x5_f32": 2, "dilate3x3": 1,
          "erode3x3": 1, "median3x3": 1}

# Nodes whose results are a few values rather than an image (Table 2).
GLOBAL_OPS = ("histogram", "min_max", "min_max_loc", "mean_std_dev")

_lib = None


def build(force: bool = False) -> str:
    """Compile the reference with gcc (-O2, no fast-math).  Returns the path."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-std=c99", "-fno-fast-math", "-o", tmp, _SRC,
                               "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _c(a: np.ndarray, dtype) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=dtype)


# ---------------------------------------------------------------------------
# single-node functions (numpy in, numpy out)
# ---------------------------------------------------------------------------

def channel_extract_y(uyvy: np.ndarray) -> np.ndarray:
    """Luma plane of a UYVY frame given as an (H, 2W) byte array."""
    uyvy = _c(uyvy, np.uint8)
    h, w2 = uyvy.shape
    out = np.empty((h, w2 // 2), np.uint8)
    lib().orc_channel_extract_y(_p(uyvy), _p(out), w2 // 2, h)
    return out


def _local_u8(fn, img, border, c):
    img = _c(img, np.uint8)
    h, w = img.shape
    out = np.empty_like(img)
    getattr(lib(), fn)(_p(img), _p(out), w, h, BORDERS[border], int(c))
    return out


def gaussian3x3(img, border="replicate", c=0):
    return _local_u8("orc_gaussian3x3", img, border, c)


def gaussian5x5(img, border="replicate", c=0):
    return _local_u8("orc_gaussian5x5", img, border, c)


def box3x3(img, border="replicate", c=0):
    return _local_u8("orc_box3x3", img, border, c)


def dilate3x3(img, border="replicate", c=0):
    """Table 2 local operator, MAX over the 3x3 window."""
    return _local_u8("orc_dilate3x3", img, border, c)


def erode3x3(img, border="replicate", c=0):
    """Table 2 local operator, MIN over the 3x3 window."""
    return _local_u8("orc_erode3x3", img, border, c)


def median3x3(img, border="replicate", c=0):
    """Table 2 local operator, MEDIAN of the 3x3 window."""
    return _local_u8("orc_median3x3", img, border, c)


NONLINEAR = {"median": 0, "min": 1, "max": 2}


def nonmax(img, win=3, border="replicate", c=0):
    """Table 2 local operator NonMaxSuppression over a win x win window (win
    3 or 5) of a U8 or S16 image (see orc_nonmax)."""
    img = np.ascontiguousarray(img)
    if img.dtype not in (np.uint8, np.int16) or win not in (3, 5):
        raise ValueError("U8 or S16 input, window 3 or 5")
    out = np.empty_like(img)
    lib().orc_nonmax(_p(img), _p(out), int(img.dtype == np.int16), int(win), img.shape[1], img.shape[0],
                     BORDERS[border], int(c))
    return out


def nonlinear(img, mask, func, border="replicate", c=0):
    """Table 2 local operator: median / min / max over the window pixels
    where `mask` (odd rows x cols, at most 9x9) is nonzero."""
    img = _c(img, np.uint8)
    mask = _c((np.asarray(mask) != 0).astype(np.uint8), np.uint8)
    rows, cols = mask.shape
    if rows % 2 == 0 or cols % 2 == 0 or rows > 9 or cols > 9 or not mask.any():
        raise ValueError("mask must be odd-sized, at most 9x9, with a nonzero entry")
    out = np.empty(img.shape, np.uint8)
    lib().orc_nonlinear(_p(img), _p(mask), cols, rows, NONLINEAR[func], _p(out), img.shape[1], img.shape[0],
                        BORDERS[border], int(c))
    return out


def sobel3x3(img, border="replicate", c=0):
    img = _c(img, np.uint8)
    h, w = img.shape
    gx = np.empty((h, w), np.int16)
    gy = np.empty((h, w), np.int16)
    lib().orc_sobel3x3(_p(img), _p(gx), _p(gy), w, h, BORDERS[border], int(c))
    return gx, gy


def magnitude(gx, gy):
    gx, gy = _c(gx, np.int16), _c(gy, np.int16)
    out = np.empty_like(gx)
    lib().orc_magnitude(_p(gx), _p(gy), _p(out), gx.shape[1], gx.shape[0])
    return out


def phase(gx, gy):
    gx, gy = _c(gx, np.int16), _c(gy, np.int16)
    out = np.empty(gx.shape, np.uint8)
    lib().orc_phase(_p(gx), _p(gy), _p(out), gx.shape[1], gx.shape[0])
    return out


def threshold(img, thresh, true_v=255, false_v=0):
    if img.dtype == np.uint8:
        kind, img = 0, _c(img, np.uint8)
    elif img.dtype == np.int16:
        kind, img = 1, _c(img, np.int16)
    else:
        kind, img = 2, _c(img, np.float64)
    out = np.empty(img.shape, np.uint8)
    lib().orc_threshold(_p(img), kind, ctypes.c_double(thresh), int(true_v), int(false_v), _p(out), img.shape[1],
                        img.shape[0])
    return out


def _kind(a):
    return 0 if a.dtype == np.uint8 else 1


def add(a, b, out_dtype="u8", policy="saturate"):
    a = a if a.dtype in (np.uint8, np.int16) else a.astype(np.int16)
    b = b if b.dtype in (np.uint8, np.int16) else b.astype(np.int16)
    a, b = np.ascontiguousarray(a), np.ascontiguousarray(b)
    ko = 0 if out_dtype == "u8" else 1
    out = np.empty(a.shape, np.uint8 if ko == 0 else np.int16)
    lib().orc_add(_p(a), _kind(a), _p(b), _kind(b), _p(out), ko, 0 if policy == "saturate" else 1, a.shape[1],
                  a.shape[0])
    return out


def multiply_f64(a, b):
    a, b = _c(a, np.int16), _c(b, np.int16)
    out = np.empty(a.shape, np.float64)
    lib().orc_multiply_f64(_p(a), _p(b), _p(out), a.shape[1], a.shape[0])
    return out


def box5x5_f64(img, border="replicate", c=0.0):
    img = _c(img, np.float64)
    out = np.empty_like(img)
    lib().orc_box5x5_f64(_p(img), _p(out), img.shape[1], img.shape[0], BORDERS[border], ctypes.c_double(c))
    return out


def harris_response(sxx, syy, sxy, k=0.04):
    sxx, syy, sxy = _c(sxx, np.float64), _c(syy, np.float64), _c(sxy, np.float64)
    out = np.empty_like(sxx)
    lib().orc_harris_response(_p(sxx), _p(syy), _p(sxy), ctypes.c_double(k), _p(out), sxx.shape[1], sxx.shape[0])
    return out


def convolve(img, coeffs, scale, out_dtype="u8", border="replicate", c=0):
    img = _c(img, np.uint8)
    coeffs = _c(coeffs, np.int16)
    rows, cols = coeffs.shape
    if rows % 2 == 0 or cols % 2 == 0:
        raise ValueError("mask dimensions must be odd")
    ko = 0 if out_dtype == "u8" else 1
    out = np.empty(img.shape, np.uint8 if ko == 0 else np.int16)
    lib().orc_convolve(_p(img), _p(coeffs), cols, rows, int(scale), _p(out), ko, img.shape[1], img.shape[0],
                       BORDERS[border], int(c))
    return out


# ---------------------------------------------------------------------------
# node-by-node graph executor
# ---------------------------------------------------------------------------

@dataclass
class Node:
    op: str
    inputs: list
    outputs: list
    border: str = "replicate"
    constant: float = 0
    params: dict = field(default_factory=dict)


class Graph:
    """A list of nodes over named images.  Names that are not produced by any
    node are graph inputs and must be supplied to :func:`run`."""

    def __init__(self):
        self.nodes: list[Node] = []

    def add(self, op, inputs, outputs, border="replicate", constant=0, **params):
        self.nodes.append(Node(op, list(inputs), list(outputs), border, constant, params))
        return self


def _topo(nodes):
    produced = {o: i for i, n in enumerate(nodes) for o in n.outputs if o is not None}
    order, state = [], {}

    def visit(i):
        if state.get(i) == 2:
            return
        if state.get(i) == 1:
            raise ValueError("graph has a cycle")
        state[i] = 1
        for name in nodes[i].inputs:
            if name in produced:
                visit(produced[name])
        state[i] = 2
        order.append(i)

    for i in range(len(nodes)):
        visit(i)
    return [nodes[i] for i in order]


def _run_node(n: Node, env: dict):
    ins = [env[name] for name in n.inputs]
    b, c, p = n.border, n.constant, n.params
    if n.op == "channel_extract_y":
        res = [channel_extract_y(ins[0])]
    elif n.op == "gaussian3x3":
        res = [gaussian3x3(ins[0], b, c)]
    elif n.op == "gaussian5x5":
        res = [gaussian5x5(ins[0], b, c)]
    elif n.op == "box3x3":
        res = [box3x3(ins[0], b, c)]
    elif n.op == "dilate3x3":
        res = [dilate3x3(ins[0], b, c)]
    elif n.op == "erode3x3":
        res = [erode3x3(ins[0], b, c)]
    elif n.op == "median3x3":
        res = [median3x3(ins[0], b, c)]
    elif n.op == "sobel3x3":
        res = list(sobel3x3(ins[0], b, c))
    elif n.op == "magnitude":
        res = [magnitude(ins[0], ins[1])]
    elif n.op == "phase":
        res = [phase(ins[0], ins[1])]
    elif n.op == "threshold":
        res = [threshold(ins[0], p["thresh"], p.get("true_v", 255), p.get("false_v", 0))]
    elif n.op == "add":
        res = [add(ins[0], ins[1], p.get("out_dtype", "u8"), p.get("policy", "saturate"))]
    elif n.op == "multiply_f32":
        res = [multiply_f64(ins[0], ins[1])]
    elif n.op == "box5x5_f32":
        res = [box5x5_f64(ins[0], b, float(c))]
    elif n.op == "harris_response":
        res = [harris_response(ins[0], ins[1], ins[2], p.get("k", 0.04))]
    elif n.op == "convolve":
        res = [convolve(ins[0], p["coeffs"], p["scale"], p.get("out_dtype", "u8"), b, c)]
    elif n.op == "nonlinear":
        res = [nonlinear(ins[0], p["mask"], p["func"], b, c)]
    elif n.op == "nonmax":
        res = [nonmax(ins[0], p.get("win", 3), b, c)]
    elif n.op == "custom_point":
        from . import custom
        res = [custom.evaluate(p["expr"], ins, p["out_dtype"])]
    elif n.op == "custom_local":
        from . import custom
        res = [custom.evaluate_local(p["expr"], ins[0], p["out_dtype"], b, c)]
    elif n.op == "histogram":
        from . import globalops
        res = [globalops.histogram(ins[0], p["bins"], p.get("offset", 0), p.get("range", 256))]
    elif n.op == "min_max":
        from . import globalops
        res = [globalops.min_max(ins[0])]
    elif n.op == "min_max_loc":
        from . import globalops
        mn, mx, cmin, cmax, lmin, lmax = globalops.min_max_loc(ins[0])
        res = [(mn, mx, cmin, cmax), (lmin, lmax)]
    elif n.op == "mean_std_dev":
        from . import globalops
        res = [globalops.mean_std_dev(ins[0])]
    elif n.op == "equalize_hist":
        from . import globalops
        res = [globalops.equalize_hist(ins[0])]
    else:
        raise ValueError("unknown op " + n.op)
    for name, val in zip(n.outputs, res):
        if name is not None:
            env[name] = val


def run(graph: Graph, inputs: dict) -> dict:
    """Execute every node of ``graph`` over full images.  Returns a dict with
    the inputs and every produced image (intermediates included)."""
    env = dict(inputs)
    for n in _topo(graph.nodes):
        _run_node(n, env)
    return env


def _radius(n: Node) -> tuple:
    if n.op in ("convolve", "nonlinear"):
        rows, cols = np.asarray(n.params["coeffs" if n.op == "convolve" else "mask"]).shape
        return cols // 2, rows // 2
    if n.op == "nonmax":
        r = n.params.get("win", 3) // 2
        return r, r
    if n.op == "custom_local":
        import ast
        from . import custom
        rx = ry = 0
        for node in ast.walk(custom.check(n.params["expr"], 1, True, local=True)):
            if isinstance(node, ast.Subscript):
                dx, dy = custom._offset(node)
                rx, ry = max(rx, abs(dx)), max(ry, abs(dy))
        return rx, ry
    r = RADIUS.get(n.op, 0)
    return r, r


def valid_masks(graph: Graph, shapes: dict) -> dict:
    """Pixels whose value is specified.  A local node with UNDEFINED border
    leaves unspecified every output pixel whose window leaves the image; any
    node's output is unspecified where a window pixel it reads is unspecified.
    ``shapes`` gives (H, W) of the graph inputs (UYVY given in pixels)."""
    env = {k: np.ones(s, bool) for k, s in shapes.items()}
    for n in _topo(graph.nodes):
        if n.op in GLOBAL_OPS:  # results are values, not images
            continue
        ins = [env[name] for name in n.inputs]
        rx, ry = _radius(n)
        h, w = ins[0].shape
        acc = np.ones((h, w), bool)
        for m in ins:
            if rx == 0 and ry == 0:
                acc &= m
                continue
            pad = np.pad(m, ((ry, ry), (rx, rx)), constant_values=(n.border != "undefined"))
            for j in range(2 * ry + 1):
                for i in range(2 * rx + 1):
                    acc &= pad[j:j + h, i:i + w]
        for name in n.outputs:
            if name is not None:
                env[name] = acc.copy()
    return env
