"""Oracle for the best-view snapshot (TEST INFRASTRUCTURE ONLY).

Section III-C picks, among views of the volume turning about Z, the rendered
image with the highest Shannon entropy (Eq. 2) of its normalised histogram.
Readings of points the paper leaves open (also listed in the design notes):
  * the image is the rendered RGBA frame (background already composited);
    each RGB channel becomes an 8-bit code q = floor(255 clamp(c, 0, 1) + 0.5)
    evaluated in FP32 (the precision of the frames), first the product, then
    the sum;
  * the grey value of a pixel is the integer BT.601 luminance
    Y = (77 q_r + 150 q_g + 29 q_b + 128) >> 8, so m = 256 bins;
  * H = -sum_i p_i log2 p_i over the non-empty bins, p_i = count_i / pixels,
    in FP64;
  * the best view is the first view of maximal entropy.
"""
from __future__ import annotations

import numpy as np


def channel_codes(c: np.ndarray) -> np.ndarray:
    """8-bit codes of FP32 channel values (clamp, scale, add one half, floor), all in FP32."""
    c = np.asarray(c, dtype=np.float32)
    x = np.minimum(np.maximum(c, np.float32(0.0)), np.float32(1.0))
    y = (x * np.float32(255.0)).astype(np.float32) + np.float32(0.5)
    return np.floor(y.astype(np.float32)).astype(np.int64)


def grey_codes(rgba: np.ndarray) -> np.ndarray:
    """Grey value 0..255 of every pixel of frames [..., 4] (RGB used, alpha ignored)."""
    q = channel_codes(rgba[..., :3])
    return (77 * q[..., 0] + 150 * q[..., 1] + 29 * q[..., 2] + 128) >> 8


def histograms(rgba: np.ndarray) -> np.ndarray:
    """[V][256] counts of the grey values of frames [V][H][W][4]."""
    g = grey_codes(rgba)
    V = g.shape[0]
    return np.stack([np.bincount(g[v].ravel(), minlength=256) for v in range(V)]).astype(np.int64)


def entropy(counts: np.ndarray) -> float:
    """Eq. 2: Shannon entropy in bits of the normalised histogram `counts`."""
    counts = np.asarray(counts, dtype=np.float64)
    n = counts.sum()
    p = counts[counts > 0] / n
    return float(-(p * np.log2(p)).sum())


def best_view(rgba: np.ndarray):
    """(index of the first view of maximal entropy, entropies of all views)."""
    H = [entropy(h) for h in histograms(rgba)]
    return int(np.argmax(H)), np.array(H)
