"""Oracle for the reduction half of the preview path (TEST INFRASTRUCTURE ONLY).

Plain NumPy / Python, exact integer arithmetic (or FP64 where the paper's
algorithm is itself floating point).  No blocking, fusion or reordering beyond
what each definition states.

Readings of points where the paper is silent or ambiguous (each is also listed
in the design notes):
  * "top 3 slices" (Section III-D) are slices z in [z0, z0 + 3) of the stored
    volume, z0 = 0 by default.
  * The "undesirable" bins (Section III-D) are every bin that occurs at least
    once in the top-slice histogram.
  * The threshold (Section III-A) for the 16-bit volume is the first valley
    above the air peak of the box-smoothed histogram S (radius r = 32): p is
    the global maximum of S (lowest bin on ties); b* is the first bin above p
    at which S has fallen to at most half its peak (2 S[b] <= S[p]) and then
    rises (S[b+1] > S[b]); T is the first bin of the plateau of S that ends at
    b*.  With no such bin the threshold is 65535.  The half-height condition
    keeps counting noise on the flat top of a broad air peak from passing
    for a valley.
  * Removed voxels become 0; kept voxels keep their grey value.
  * Pyramid level k is the round-half-up mean over the full 2^k cube, taken
    from the exact integer box sum with zero padding past the volume's end
    (never from the previous rounded level).
  * Slicemap atlas (Section III, the slicemap format of the cited prior work):
    slice z occupies tile (z mod tiles_x, z div tiles_x), row-major, unused
    tiles are 0; the 8-bit form is min(255, (L + 128) >> 8).
  * Otsu (Algorithm 1): maximise the between-class variance w_a w_b (mu_a -
    mu_b)^2 over T with class a = bins [0, T) and class b = bins [T, B-1]
    (the last bin included), strictly-greater update so ties keep the lowest
    T, empty classes are not candidates; evaluated in FP64 in exactly the
    order written in Algorithm 1.
  * ITS (Algorithm 2, whose printed update of r is garbled): the isodata
    iteration T <- floor((mu_1 + mu_2) / 2), classes as for Otsu, stopping
    when T repeats (so mu_1 and mu_2 stay constant); an empty class stops with
    the current T; FP64 evaluation.  The start is the middle of the occupied
    dynamic range, T = (b_min + b_max + 1) div 2 over the non-empty bins
    (the paper starts in the middle of an 8-bit range that its data fills;
    a 16-bit scan fills only part of its range).
"""
from __future__ import annotations

import numpy as np

NBINS = 65536


# ---------------------------------------------------------------- histogram
def histogram(vol: np.ndarray, z0: int = 0, nz_range: int | None = None) -> np.ndarray:
    """Section III-D: H[b] = number of voxels of value b in slices [z0, z0+nz_range)."""
    vol = np.asarray(vol)
    assert vol.dtype == np.uint16 and vol.ndim == 3
    nz = vol.shape[0]
    if nz_range is None:
        nz_range = nz - z0
    slab = vol[z0:z0 + nz_range]
    return np.bincount(slab.ravel(), minlength=NBINS).astype(np.uint64)


# ----------------------------------------------------------- threshold rules
def smoothed(H: np.ndarray, r: int) -> np.ndarray:
    """S[b] = sum of H[k] for k in [max(0, b-r), min(B-1, b+r)], exact uint64."""
    H = np.asarray(H, dtype=np.uint64)
    B = H.shape[0]
    c = np.zeros(B + 1, dtype=np.uint64)
    np.cumsum(H, out=c[1:])
    b = np.arange(B)
    lo = np.maximum(b - r, 0)
    hi = np.minimum(b + r, B - 1)
    return c[hi + 1] - c[lo]


def valley_threshold(H: np.ndarray, r: int = 32) -> int:
    """First valley above the air peak of the smoothed histogram (reading above)."""
    S = smoothed(H, r)
    B = S.shape[0]
    p = int(np.argmax(S))
    bstar = None
    for b in range(p + 1, B - 1):
        if 2 * int(S[b]) <= int(S[p]) and S[b + 1] > S[b]:
            bstar = b
            break
    if bstar is None:
        return B - 1
    T = bstar
    while T - 1 > p and S[T - 1] == S[bstar]:
        T -= 1
    return T


def otsu_threshold(H: np.ndarray) -> int:
    """Algorithm 1 (Otsu), FP64: maximise w_a * w_b * (U_a - U_b)^2."""
    H = np.asarray(H, dtype=np.uint64)
    B = H.shape[0]
    N = int(H.sum())
    best_T, best = 0, 0.0
    n_a = 0
    s_a = 0
    s_tot = int(np.dot(np.arange(B, dtype=np.uint64), H))
    for T in range(B):
        # class a = [0, T): add bin T-1 before evaluating T
        if T > 0:
            n_a += int(H[T - 1])
            s_a += (T - 1) * int(H[T - 1])
        n_b = N - n_a
        if n_a == 0 or n_b == 0:
            continue
        s_b = s_tot - s_a
        w_a = float(n_a) / float(N)
        w_b = float(n_b) / float(N)
        u_a = float(s_a) / float(n_a)
        u_b = float(s_b) / float(n_b)
        d = u_a - u_b
        sigma = (w_a * w_b) * (d * d)
        if sigma > best:
            best, best_T = sigma, T
    return best_T


def its_threshold(H: np.ndarray, max_iter: int = 1000):
    """Algorithm 2 (ITS / isodata), FP64.  Returns (T, iterations)."""
    H = np.asarray(H, dtype=np.uint64)
    B = H.shape[0]
    nz = np.nonzero(H)[0]
    if len(nz) == 0:
        return 0, 0
    T = (int(nz[0]) + int(nz[-1]) + 1) // 2
    it = 0
    while it < max_iter:
        it += 1
        n1 = int(H[:T].sum())
        n2 = int(H[T:].sum())
        if n1 == 0 or n2 == 0:
            return T, it
        s1 = int(np.dot(np.arange(T, dtype=np.uint64), H[:T]))
        s2 = int(np.dot(np.arange(T, B, dtype=np.uint64), H[T:]))
        mu1 = float(s1) / float(n1)
        mu2 = float(s2) / float(n2)
        Tn = int(np.floor((mu1 + mu2) / 2.0))
        if Tn == T:
            return T, it
        T = Tn
    return T, it


def keep_bits(T: int, H_top: np.ndarray | None = None) -> np.ndarray:
    """keep[b] = (b >= T) and (H_top[b] == 0); packed, bin b -> bit b%32 of word b//32."""
    b = np.arange(NBINS)
    keep = b >= T
    if H_top is not None:
        keep &= np.asarray(H_top) == 0
    return pack_bits(keep)


def pack_bits(keep: np.ndarray) -> np.ndarray:
    keep = np.asarray(keep, dtype=bool).reshape(NBINS // 32, 32)
    w = (keep.astype(np.uint64) << np.arange(32, dtype=np.uint64)).sum(axis=1)
    return w.astype(np.uint32)


def unpack_bits(bits: np.ndarray) -> np.ndarray:
    bits = np.asarray(bits, dtype=np.uint32)
    return ((bits[:, None] >> np.arange(32, dtype=np.uint32)) & 1).astype(bool).ravel()


# ------------------------------------------------------------------ pyramid
def apply_keep(vol: np.ndarray, bits: np.ndarray | None) -> np.ndarray:
    """Thresholding / histogram filtering (Sections III-A, III-D): f = keep[v] ? v : 0."""
    vol = np.asarray(vol)
    if bits is None:
        return vol.copy()
    keep = unpack_bits(bits)
    return np.where(keep[vol], vol, np.uint16(0)).astype(np.uint16)


def level_dims(nx: int, ny: int, nz: int, k: int):
    d = 1 << k
    return (-(-nx // d), -(-ny // d), -(-nz // d))


def box_sums(f: np.ndarray, k: int) -> np.ndarray:
    """S_k[z][y][x] = sum of f over the 2^k cube at 2^k (x, y, z), zero padded, int64."""
    nz, ny, nx = f.shape
    d = 1 << k
    mx, my, mz = level_dims(nx, ny, nz, k)
    pad = np.zeros((mz * d, my * d, mx * d), dtype=np.int64)
    pad[:nz, :ny, :nx] = f
    return pad.reshape(mz, d, my, d, mx, d).sum(axis=(1, 3, 5))


def level_from_sums(S: np.ndarray, k: int) -> np.ndarray:
    """L_k = (S_k + 2^(3k-1)) >> 3k, the round-half-up mean over the 8^k box."""
    S = np.asarray(S, dtype=np.int64)
    return ((S + (1 << (3 * k - 1))) >> (3 * k)).astype(np.uint16)


def pyramid(vol: np.ndarray, bits: np.ndarray | None, n_levels: int):
    """Levels 1..n_levels of the filtered volume, each from its own exact sums."""
    f = apply_keep(vol, bits)
    return [level_from_sums(box_sums(f, k), k) for k in range(1, n_levels + 1)]


def box_sum_at(vol: np.ndarray, bits: np.ndarray | None, k: int, zyx) -> np.ndarray:
    """S_k at the given level-k voxel positions, summed directly from the volume."""
    keep = None if bits is None else unpack_bits(bits)
    d = 1 << k
    out = np.zeros(len(zyx), dtype=np.int64)
    for i, (z, y, x) in enumerate(zyx):
        blk = np.asarray(vol[z * d:(z + 1) * d, y * d:(y + 1) * d, x * d:(x + 1) * d])
        if keep is not None:
            blk = np.where(keep[blk], blk, 0)
        out[i] = int(blk.astype(np.int64).sum())
    return out


# ----------------------------------------------------------------- slicemap
def slicemap(L: np.ndarray, tiles_x: int, tiles_y: int, out_bits: int = 16) -> np.ndarray:
    """Atlas pixel (tx*nx + x, ty*ny + y) = L[z][y][x] with z = ty*tiles_x + tx."""
    nz, ny, nx = L.shape
    assert tiles_x * tiles_y >= nz
    A = np.zeros((tiles_y * ny, tiles_x * nx), dtype=np.uint16)
    for z in range(nz):
        ty, tx = divmod(z, tiles_x)
        A[ty * ny:(ty + 1) * ny, tx * nx:(tx + 1) * nx] = L[z]
    if out_bits == 8:
        A = np.minimum(255, (A.astype(np.int64) + 128) >> 8).astype(np.uint8)
    return A
