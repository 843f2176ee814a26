"""Oracle for user-defined point nodes (custom OpenVX kernels, Section 5.1).

TEST INFRASTRUCTURE ONLY (see the package docstring).  The paper lets users
add their own kernels to a graph as generic nodes, analysed and fused like
the built-in ones.  Here a user point kernel is an arithmetic expression over
up to three input images ``a``, ``b``, ``c``; this module evaluates it over
whole images, independently of the GPU library (its own parser: Python's
``ast`` restricted to the grammar below).

Grammar: numbers, ``a``/``b``/``c``, unary ``-``, binary ``+ - * /`` with the
usual precedence and parentheses, and the functions ``min(x, y)``,
``max(x, y)``, ``abs(x)``, ``clamp(x, lo, hi)`` (= min(max(x, lo), hi)),
``gt(x, y)`` (1 where x > y, else 0), ``sel(p, x, y)`` (x where p != 0, else
y) and ``sqrt(x)`` (float kernels only).

A user local kernel has one input ``a`` and may also read it at offsets
``a[dx, dy]`` (integers, |dx|, |dy| <= 2; ``a`` alone is ``a[0, 0]``); the
positions outside the image follow the node's border mode.

Integer kernels (every input U8/S16, output U8/S16) compute in 32-bit two's
complement: + - * and negation wrap modulo 2^32, / truncates toward zero,
x / 0 = 0 and the one overflowing quotient (-2^31) / (-1) wraps to -2^31.
Literals are integers that fit 32 bits.  The result is saturated to the
output type.  Float kernels (some input F32; the output must then be F32)
compute in real arithmetic, here float64; IEEE division and square root.
"""
from __future__ import annotations

import ast

import numpy as np

FUNCS = {"min": 2, "max": 2, "abs": 1, "clamp": 3, "gt": 2, "sel": 3, "sqrt": 1}
INPUTS = ("a", "b", "c")


def _wrap(x):
    return ((x + 2 ** 31) % 2 ** 32) - 2 ** 31


def _offset(n):
    """(dx, dy) of a subscript a[dx, dy] with integer literals in [-2, 2]."""
    sl = n.slice
    if not isinstance(sl, ast.Tuple) or len(sl.elts) != 2:
        raise ValueError("a[dx, dy] takes two offsets")
    out = []
    for e in sl.elts:
        neg = isinstance(e, ast.UnaryOp) and isinstance(e.op, ast.USub)
        v = e.operand if neg else e
        if not isinstance(v, ast.Constant) or isinstance(v.value, bool) or not isinstance(v.value, int):
            raise ValueError("offsets are integer literals")
        k = -v.value if neg else v.value
        if not -2 <= k <= 2:
            raise ValueError("offsets within -2..2")
        out.append(k)
    return tuple(out)


def check(expr: str, nin: int, is_float: bool, local: bool = False):
    """Raise ValueError unless ``expr`` is in the grammar for ``nin`` inputs
    (a local kernel: one input, offsets allowed)."""
    try:
        tree = ast.parse(expr, mode="eval")
    except SyntaxError as e:
        raise ValueError("syntax error: %s" % e) from None

    def walk(n):
        if isinstance(n, ast.BinOp):
            if not isinstance(n.op, (ast.Add, ast.Sub, ast.Mult, ast.Div)):
                raise ValueError("operator not allowed")
            walk(n.left)
            walk(n.right)
        elif isinstance(n, ast.UnaryOp):
            if not isinstance(n.op, ast.USub):
                raise ValueError("unary operator not allowed")
            walk(n.operand)
        elif isinstance(n, ast.Call):
            if not isinstance(n.func, ast.Name) or n.func.id not in FUNCS or n.keywords:
                raise ValueError("unknown function")
            if len(n.args) != FUNCS[n.func.id]:
                raise ValueError("wrong argument count")
            if n.func.id == "sqrt" and not is_float:
                raise ValueError("sqrt needs a float kernel")
            for x in n.args:
                walk(x)
        elif isinstance(n, ast.Subscript):
            if not local or not isinstance(n.value, ast.Name) or n.value.id != "a":
                raise ValueError("offsets only on input a of a local kernel")
            _offset(n)
        elif isinstance(n, ast.Name):
            if n.id not in INPUTS[:nin]:
                raise ValueError("unknown name %s" % n.id)
        elif isinstance(n, ast.Constant):
            if isinstance(n.value, bool) or not isinstance(n.value, (int, float)):
                raise ValueError("bad literal")
            if not is_float and (not isinstance(n.value, int) or not -2 ** 31 <= n.value < 2 ** 31):
                raise ValueError("integer kernels take 32-bit integer literals")
        else:
            raise ValueError("construct not allowed: %s" % type(n).__name__)

    walk(tree.body)
    return tree.body


_PAD = {"replicate": "edge", "undefined": "edge", "mirror": "reflect", "repeat": "wrap"}


def evaluate_local(expr: str, img: np.ndarray, out_dtype, border="replicate", c=0) -> np.ndarray:
    """A user local kernel over one image: every a[dx, dy] reads the image
    shifted by (dx, dy), positions outside it taken by the border mode
    (numpy's edge / reflect / wrap padding for REPLICATE / MIRROR / REPEAT,
    the constant for CONSTANT; UNDEFINED as REPLICATE, its border pixels
    being unspecified)."""
    f32_out = np.dtype(out_dtype).kind == "f"
    is_float = img.dtype.kind == "f" or f32_out
    tree = check(expr, 1, is_float, local=True)
    h, w = img.shape
    pad = img
    for axis, n in ((0, h), (1, w)):
        widths = ((2, 2), (0, 0)) if axis == 0 else ((0, 0), (2, 2))
        if border == "constant":
            pad = np.pad(pad, widths, mode="constant", constant_values=c)
        elif border == "mirror" and n == 1:  # a one-pixel axis repeats its pixel
            pad = np.pad(pad, widths, mode="edge")
        else:
            pad = np.pad(pad, widths, mode=_PAD[border])

    def shifted(dx, dy):
        return pad[2 + dy:2 + dy + h, 2 + dx:2 + dx + w]

    offs = {}

    def walk(n):
        if isinstance(n, ast.Subscript):
            offs[id(n)] = _offset(n)
        for ch in ast.iter_child_nodes(n):
            walk(ch)

    walk(tree)

    class Sub(ast.NodeTransformer):
        def visit_Subscript(self, n):
            dx, dy = offs[id(n)]
            return ast.copy_location(ast.Name(id="w_%d_%d" % (dx + 2, dy + 2), ctx=ast.Load()), n)

    names = {}
    for dx in range(-2, 3):
        for dy in range(-2, 3):
            names["w_%d_%d" % (dx + 2, dy + 2)] = shifted(dx, dy)
    return _run(Sub().visit(tree), {"a": img, **names}, shape=img.shape, is_float=is_float, out_dtype=out_dtype)


def evaluate(expr: str, inputs: list, out_dtype) -> np.ndarray:
    """Evaluate ``expr`` over the input images (numpy arrays of one shape:
    uint8 / int16, or a float type standing for F32).  ``out_dtype``:
    np.uint8, np.int16, or a float type (F32 output, computed in float64)."""
    f32_out = np.dtype(out_dtype).kind == "f"
    is_float = any(x.dtype.kind == "f" for x in inputs) or f32_out
    if is_float and not f32_out:
        raise ValueError("a float kernel has an F32 output")
    tree = check(expr, len(inputs), is_float)
    return _run(tree, {INPUTS[i]: x for i, x in enumerate(inputs)}, inputs[0].shape, is_float, out_dtype)


def _run(tree, images: dict, shape, is_float: bool, out_dtype):
    env = {k: (x.astype(np.float64) if is_float else x.astype(np.int64)) for k, x in images.items()}

    def ev(n):
        if isinstance(n, ast.Constant):
            return np.full(shape, n.value, np.float64 if is_float else np.int64)
        if isinstance(n, ast.Name):
            return env[n.id]
        if isinstance(n, ast.UnaryOp):
            v = -ev(n.operand)
            return v if is_float else _wrap(v)
        if isinstance(n, ast.BinOp):
            x, y = ev(n.left), ev(n.right)
            if isinstance(n.op, ast.Add):
                r = x + y
            elif isinstance(n.op, ast.Sub):
                r = x - y
            elif isinstance(n.op, ast.Mult):
                r = x * y
            elif is_float:
                with np.errstate(divide="ignore", invalid="ignore"):
                    r = x / y
            else:  # truncating division on the exact int64 values, x / 0 = 0
                q = np.abs(x) // np.where(y == 0, 1, np.abs(y))
                r = np.where(y == 0, 0, np.where((x < 0) != (y < 0), -q, q))
            return r if is_float else _wrap(r)
        f = n.func.id
        args = [ev(x) for x in n.args]
        if f == "min":
            return np.minimum(args[0], args[1])
        if f == "max":
            return np.maximum(args[0], args[1])
        if f == "abs":
            return np.abs(args[0]) if is_float else _wrap(np.abs(args[0]))
        if f == "clamp":
            return np.minimum(np.maximum(args[0], args[1]), args[2])
        if f == "gt":
            return (args[0] > args[1]).astype(args[0].dtype)
        if f == "sel":
            return np.where(args[0] != 0, args[1], args[2])
        with np.errstate(invalid="ignore"):
            return np.sqrt(args[0])

    r = ev(tree)
    if is_float:
        return r
    info = np.iinfo(out_dtype)
    return np.clip(r, info.min, info.max).astype(out_dtype)
