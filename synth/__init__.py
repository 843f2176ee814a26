"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module only draws pixels, shapes and arrival times.  It holds none of the
image-processing arithmetic: neither the library nor the CPU reference imports
anything from it, and it imports neither of them.

The paper evaluates on unspecified camera images of 1024x1024, 2048x2048 and
1020x1020 pixels (Section 6).  No public dataset is involved, so every input
here is generated from a seed with ``numpy.random.default_rng`` (PCG64).
"""
from __future__ import annotations

import numpy as np

# Row pitch alignment (bytes) used for every device-side image buffer.
PITCH_ALIGN = 64

# The image kinds used by the workloads.
GRAPH_TYPES = ("sobel_edge", "harris", "gauss5")
SERVE_TYPES = ("sobel_edge", "harris", "uyvy_gauss5")
SERVE_SIZES = ((640, 480), (1280, 720), (1920, 1080), (3840, 2160))


def pitch_for(width_bytes: int, align: int = PITCH_ALIGN) -> int:
    """Smallest multiple of ``align`` that holds ``width_bytes``."""
    return max(align, (int(width_bytes) + align - 1) // align * align)


def edge_image(w: int, h: int, seed: int = 0) -> np.ndarray:
    """Uniform U8 noise plus 8 flat filled rectangles (the edge-graph input).

    Rectangles: top-left uniform in the image, sides uniform in [W/16, W/4] and
    [H/16, H/4], fill level uniform in [0, 255], clipped to the image.
    """
    rng = np.random.default_rng(seed)
    img = rng.integers(0, 256, size=(h, w), dtype=np.uint8)
    for _ in range(8):
        x0 = int(rng.integers(0, w))
        y0 = int(rng.integers(0, h))
        rw = int(rng.integers(max(1, w // 16), max(1, w // 4) + 1))
        rh = int(rng.integers(max(1, h // 16), max(1, h // 4) + 1))
        v = int(rng.integers(0, 256))
        img[y0:y0 + rh, x0:x0 + rw] = v
    return img


def corner_image(w: int, h: int, seed: int = 0) -> np.ndarray:
    """Smooth random blobs plus checkerboard patches (the corner-graph input).

    Background 128; 64 Gaussian blobs with centres uniform in the image,
    sigma uniform in [10, 60] px and amplitude uniform in [-80, 80]; then 16
    checkerboard patches with cells of 8..32 px, 2..4 cells per side and
    levels 40 / 215.  Rounded and clipped to U8.
    """
    rng = np.random.default_rng(seed)
    yy, xx = np.mgrid[0:h, 0:w].astype(np.float64)
    acc = np.full((h, w), 128.0)
    for _ in range(64):
        cx = rng.uniform(0, w)
        cy = rng.uniform(0, h)
        sg = rng.uniform(10, 60)
        amp = rng.uniform(-80, 80)
        # evaluate only inside a 4-sigma window to keep large images cheap
        x0, x1 = int(max(0, cx - 4 * sg)), int(min(w, cx + 4 * sg + 1))
        y0, y1 = int(max(0, cy - 4 * sg)), int(min(h, cy + 4 * sg + 1))
        if x0 >= x1 or y0 >= y1:
            continue
        sx = xx[y0:y1, x0:x1] - cx
        sy = yy[y0:y1, x0:x1] - cy
        acc[y0:y1, x0:x1] += amp * np.exp(-(sx * sx + sy * sy) / (2 * sg * sg))
    img = np.clip(np.rint(acc), 0, 255).astype(np.uint8)
    for _ in range(16):
        cell = int(rng.integers(8, 33))
        nx = int(rng.integers(2, 5))
        ny = int(rng.integers(2, 5))
        x0 = int(rng.integers(0, max(1, w - cell)))
        y0 = int(rng.integers(0, max(1, h - cell)))
        for j in range(ny):
            for i in range(nx):
                lvl = 215 if (i + j) % 2 else 40
                img[y0 + j * cell:y0 + (j + 1) * cell, x0 + i * cell:x0 + (i + 1) * cell] = lvl
    return img


def uyvy_image(w: int, h: int, seed: int = 0) -> np.ndarray:
    """UYVY 4:2:2 frame as an (H, 2W) byte array: U Y0 V Y1 per pixel pair.

    The luma plane is ``edge_image(w, h, seed)``; chroma bytes are uniform.
    ``w`` must be even.
    """
    if w % 2:
        raise ValueError("UYVY width must be even")
    rng = np.random.default_rng(seed + 7919)
    out = np.empty((h, 2 * w), dtype=np.uint8)
    out[:, 1::2] = edge_image(w, h, seed)
    out[:, 0::2] = rng.integers(0, 256, size=(h, w), dtype=np.uint8)
    return out


def frame_recipe(i: int, n_bases: int = 4):
    """Frame i of a multi-frame workload: (seed of its base image, byte it is
    XORed with).  Frames cycle over ``n_bases`` seeded ``edge_image`` bases,
    and each cycle XORs a different byte into every pixel, so all frames are
    distinct buffers with the statistics of the bases."""
    return i % n_bases, (i // n_bases) * 37 % 256


def recipe_frame(w: int, h: int, i: int, n_bases: int = 4) -> np.ndarray:
    """Host copy of frame i of ``frame_recipe`` (the base image XOR its byte)."""
    seed, x = frame_recipe(i, n_bases)
    return edge_image(w, h, seed=seed) ^ np.uint8(x)


def uniform_u8(w: int, h: int, seed: int = 0) -> np.ndarray:
    return np.random.default_rng(seed).integers(0, 256, size=(h, w), dtype=np.uint8)


def uniform_s16(w: int, h: int, seed: int = 0, lo: int = -32768, hi: int = 32767) -> np.ndarray:
    return np.random.default_rng(seed).integers(lo, hi + 1, size=(h, w), dtype=np.int16)


def padded(img: np.ndarray, align: int = PITCH_ALIGN, seed: int = 12345) -> np.ndarray:
    """Copy ``img`` (H, W[*bpp]) into an (H, pitch) byte-compatible buffer whose
    row padding is filled with random bytes, so that any read of the padding
    shows up as a wrong result.  Returns the padded array (same dtype)."""
    h = img.shape[0]
    row_bytes = img.shape[1] * img.itemsize
    pitch = pitch_for(row_bytes, align)
    assert pitch % img.itemsize == 0
    rng = np.random.default_rng(seed)
    buf = rng.integers(0, 256, size=(h, pitch), dtype=np.uint8).view(img.dtype)
    buf[:, :img.shape[1]] = img
    return buf


def batch_shapes(n: int = 256, seed: int = 0):
    """Shapes and graph kinds of the mixed batch: W ~ U{320..4096},
    H ~ U{240..2160}, kind ~ U{sobel_edge, harris, gauss5}.  Image i is drawn
    with seed 1000 + i."""
    rng = np.random.default_rng(seed)
    ws = rng.integers(320, 4097, size=n)
    hs = rng.integers(240, 2161, size=n)
    ks = rng.integers(0, len(GRAPH_TYPES), size=n)
    return [(int(w), int(h), GRAPH_TYPES[int(k)], 1000 + i) for i, (w, h, k) in enumerate(zip(ws, hs, ks))]


def serving_trace(rate_hz: float, n: int, seed: int = 0):
    """Poisson arrivals at ``rate_hz``: list of (t_arrival_s, kind, w, h, seed)."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_hz, size=n)
    t = np.cumsum(gaps) - gaps[0]
    kinds = rng.integers(0, len(SERVE_TYPES), size=n)
    sizes = rng.integers(0, len(SERVE_SIZES), size=n)
    return [(float(t[i]), SERVE_TYPES[int(kinds[i])], SERVE_SIZES[int(sizes[i])][0],
             SERVE_SIZES[int(sizes[i])][1], 5000 + i) for i in range(n)]
