"""Oracle for container removal (TEST INFRASTRUCTURE ONLY).

Section III-B finds the cylindrical sample container as a circle in the top
slice with the Hough circle transform of Ioannou et al. (centres by a 2D
accumulation along gradient lines, the radius by a histogram of distances),
then discards everything outside that circle in every slice.

Readings of points the paper leaves open (also listed in the design notes):
  * the top slice is slice 0 of the stack (the same end whose first three
    slices give the top-slice histogram of Section III-D);
  * edges: the integer 3 x 3 Sobel gradient (gx, gy) of the interior pixels
    (border pixels carry none); a pixel is an edge when m2 = gx^2 + gy^2 > 0
    and m2 * 2^shift >= the slice's largest m2;
  * centre votes: every edge pixel p votes once for each pixel of the
    digital line from p against its gradient (one pixel per step along the
    gradient's major axis, the minor offset rounded half up in exact integer
    arithmetic), at the steps whose distance from p along the line lies in
    [r_min, r_max]; the container's wall is brighter than the air it holds,
    so along its inner boundary grey values rise away from the centre and
    those lines run through it; votes that leave the slice are dropped;
  * the centre is the first maximum, in row-major order, of the accumulator
    summed over (2w + 1)^2 boxes, w = max(1, r_max / 16) (cells outside the
    slice count as zero): single cells do not peak, since the gradient
    directions of a pixelated edge scatter the lines by a few pixels at the
    centre, but a box of that size collects them;
  * the radius is the first maximum (smallest radius) of the histogram of
    round(|p - c|) over the edge pixels whose gradient points away from the
    centre (g . (p - c) > 0), counted for radii in [r_min, r_max];
  * the kept disc has radius R = max(r - margin, 0) (a few voxels of margin
    leave out the partial-volume voxels of the wall) and holds the pixels
    with (x - cx)^2 + (y - cy)^2 <= R^2;
  * discarded voxels take no part in either histogram and count as zero in
    the pyramid (as voxels that thresholding removes); with no edge, no vote
    or no radius count the circle is "not found" and nothing is discarded.

The circle record is eight integers:
  [found, cx, cy, r, R, centre votes (box sum), radius count, edge pixels].
"""
from __future__ import annotations

import numpy as np

RECORD = ("found", "cx", "cy", "r", "R", "centre_votes", "radius_votes", "edges")


def sobel(s: np.ndarray):
    """Integer Sobel gradient of a 2D slice [ny][nx]; zero on the border."""
    a = np.asarray(s, dtype=np.int64)
    ny, nx = a.shape
    gx = np.zeros((ny, nx), dtype=np.int64)
    gy = np.zeros((ny, nx), dtype=np.int64)
    if nx < 3 or ny < 3:
        return gx, gy
    c = slice(1, -1)
    right = a[:-2, 2:] + 2 * a[1:-1, 2:] + a[2:, 2:]
    left = a[:-2, :-2] + 2 * a[1:-1, :-2] + a[2:, :-2]
    down = a[2:, :-2] + 2 * a[2:, 1:-1] + a[2:, 2:]
    up = a[:-2, :-2] + 2 * a[:-2, 1:-1] + a[:-2, 2:]
    gx[c, c] = right - left
    gy[c, c] = down - up
    return gx, gy


def edge_pixels(s: np.ndarray, shift: int):
    """(x, y, gx, gy) of the edge pixels in row-major order."""
    gx, gy = sobel(s)
    m2 = gx * gx + gy * gy
    G2 = int(m2.max()) if m2.size else 0
    if G2 == 0:
        e = np.zeros(0, dtype=np.int64)
        return e, e, e, e
    sel = (m2 > 0) & ((m2 << shift) >= G2)
    y, x = np.nonzero(sel)
    return x.astype(np.int64), y.astype(np.int64), gx[sel], gy[sel]


def round_sqrt(D):
    """round(sqrt(D)) with halves up for integers D >= 0 (no half ties occur)."""
    D = np.asarray(D, dtype=np.int64)
    d = np.floor(np.sqrt(D.astype(np.float64)) + 0.5).astype(np.int64)
    for _ in range(2):
        d = np.where((d > 0) & ((2 * d - 1) ** 2 > 4 * D), d - 1, d)
        d = np.where((2 * d + 1) ** 2 <= 4 * D, d + 1, d)
    return d


def line_cells(x, y, gx, gy, k):
    """Cell k (k >= 1) of the digital line from (x, y) against the gradient."""
    a, b = np.abs(gx), np.abs(gy)
    xmaj = a >= b
    gmaj, gmin = np.where(xmaj, a, b), np.where(xmaj, b, a)
    j = (2 * k * gmin + gmaj) // (2 * gmaj)          # round(k gmin / gmaj), halves up
    ox = np.where(xmaj, k, j) * np.sign(gx)
    oy = np.where(xmaj, j, k) * np.sign(gy)
    return x - ox, y - oy


def step_in_range(gx, gy, k, r_min, r_max):
    """Whether step k lies at a distance k |g| / g_major in [r_min, r_max]."""
    gmaj = np.maximum(np.abs(gx), np.abs(gy))
    d2 = k * k * (gx * gx + gy * gy)
    return (d2 >= r_min * r_min * gmaj * gmaj) & (d2 <= r_max * r_max * gmaj * gmaj)


def accumulator(s: np.ndarray, r_min: int, r_max: int, shift: int):
    """The 2D centre accumulator [ny][nx] and the edge pixels."""
    ny, nx = s.shape
    x, y, gx, gy = edge_pixels(s, shift)
    acc = np.zeros(ny * nx, dtype=np.int64)
    # the distance of step k is between k and k sqrt(2): k <= r_max suffices
    for k in range(1, r_max + 1):
        cx, cy = line_cells(x, y, gx, gy, k)
        ok = step_in_range(gx, gy, k, r_min, r_max) & (cx >= 0) & (cx < nx) & (cy >= 0) & (cy < ny)
        np.add.at(acc, cy[ok] * nx + cx[ok], 1)
    return acc.reshape(ny, nx), (x, y, gx, gy)


def peak_window(r_max: int) -> int:
    return max(1, r_max // 16)


def box_sums(acc: np.ndarray, w: int) -> np.ndarray:
    """B[y][x] = sum of acc over |y' - y| <= w, |x' - x| <= w (zero outside)."""
    ny, nx = acc.shape
    B = np.zeros_like(acc)
    for y in range(ny):
        rows = acc[max(0, y - w):y + w + 1].sum(axis=0)
        c = np.concatenate([[0], np.cumsum(rows)])
        lo = np.maximum(np.arange(nx) - w, 0)
        hi = np.minimum(np.arange(nx) + w + 1, nx)
        B[y] = c[hi] - c[lo]
    return B


def find_container(s: np.ndarray, r_min: int, r_max: int, shift: int = 4, margin: int = 2) -> np.ndarray:
    """The circle record of the slice s [ny][nx] (u16)."""
    acc, (x, y, gx, gy) = accumulator(s, r_min, r_max, shift)
    rec = np.zeros(8, dtype=np.int64)
    rec[7] = x.size
    B = box_sums(acc, peak_window(r_max))
    votes = int(B.max()) if B.size else 0
    if votes == 0:
        return rec
    i = int(np.argmax(B.ravel()))                 # first maximum, row-major
    cy, cx = divmod(i, s.shape[1])
    dx, dy = x - cx, y - cy
    out = gx * dx + gy * dy > 0
    d = round_sqrt(dx * dx + dy * dy)
    sel = out & (d >= r_min) & (d <= r_max)
    rh = np.bincount(d[sel], minlength=r_max + 1)
    if rh.size == 0 or int(rh.max()) == 0:
        rec[1], rec[2], rec[5] = cx, cy, votes
        return rec
    r = int(np.argmax(rh))                        # smallest radius on ties
    rec[:] = (1, cx, cy, r, max(r - margin, 0), votes, int(rh[r]), x.size)
    return rec


def disc_mask(nx: int, ny: int, rec) -> np.ndarray:
    """bool [ny][nx]: the pixels kept (all of them when the circle was not found)."""
    if not rec[0]:
        return np.ones((ny, nx), dtype=bool)
    X = np.arange(nx, dtype=np.int64)[None, :] - int(rec[1])
    Y = np.arange(ny, dtype=np.int64)[:, None] - int(rec[2])
    return X * X + Y * Y <= int(rec[4]) ** 2


def remove_container(vol: np.ndarray, rec) -> np.ndarray:
    """The volume with every voxel outside the disc set to 0, in every slice."""
    m = disc_mask(vol.shape[2], vol.shape[1], rec)
    return np.where(m[None, :, :], vol, 0).astype(vol.dtype)


def histogram_in_disc(vol: np.ndarray, rec, z0: int = 0, nz_range: int | None = None) -> np.ndarray:
    """H[b] = voxels of value b inside the disc among slices [z0, z0 + nz_range)."""
    if nz_range is None:
        nz_range = vol.shape[0] - z0
    m = disc_mask(vol.shape[2], vol.shape[1], rec)
    v = vol[z0:z0 + nz_range][:, m]
    return np.bincount(v.ravel().astype(np.int64), minlength=65536).astype(np.uint64)
