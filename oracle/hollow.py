"""Oracle for the hollow data preview (TEST INFRASTRUCTURE ONLY).

Section II (the data preview) asks for a reduced dataset that keeps the
object's outer geometry and drops its interior volume, giving a hollow
dataset; the paper gives no algorithm for it.

Readings (also listed in the design notes):
  * the object is the set of non-zero voxels of a thresholded volume (or of
    one of its pyramid levels), whose removed voxels are 0;
  * the shell of thickness t >= 1 is what t binary erosions of the object
    with the 6-neighbourhood (face neighbours) take away, with everything
    outside the volume counted as background: a voxel is kept when it is
    non-zero and some voxel within city-block distance t of it is zero or
    lies outside the volume;
  * kept voxels keep their grey value, every other voxel becomes 0;
  * cavities inside the object are background like any other, so their
    walls are kept too.

hollow() follows the erosion reading with SciPy's binary erosion as the
library step; tests pin it against the distance reading by brute force and
against closed forms.
"""
from __future__ import annotations

import numpy as np
from scipy import ndimage


def shell_mask(vol: np.ndarray, t: int) -> np.ndarray:
    """Boolean [nz][ny][nx]: non-zero voxels that t 6-neighbour erosions of the
    non-zero set (zero border) remove."""
    if t < 1:
        raise ValueError("thickness must be at least 1")
    obj = np.asarray(vol) != 0
    cross = ndimage.generate_binary_structure(3, 1)
    inner = ndimage.binary_erosion(obj, structure=cross, iterations=t, border_value=0)
    return obj & ~inner


def hollow(vol: np.ndarray, t: int) -> np.ndarray:
    """The volume with every voxel outside the shell of thickness t set to 0."""
    vol = np.asarray(vol)
    return np.where(shell_mask(vol, t), vol, np.zeros((), dtype=vol.dtype))


def kept_count(vol: np.ndarray, t: int) -> int:
    """Number of voxels the hollow volume keeps."""
    return int(shell_mask(vol, t).sum())
