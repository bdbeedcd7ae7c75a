"""Pins of the hollow-preview oracle to facts that do not come from it: the
city-block distance reading checked by brute force on small volumes, closed
forms for a solid box and for the octahedral shell around one empty voxel,
and invariants (grey values kept, monotone in the thickness, everything kept
once the thickness reaches half the smallest side)."""
import itertools

import numpy as np
import pytest

from oracle import hollow as HW


def _brute(vol, t):
    """Keep a non-zero voxel iff a voxel within city-block distance t is zero
    or lies outside the volume."""
    nz, ny, nx = vol.shape
    out = np.zeros_like(vol)
    offs = [d for d in itertools.product(range(-t, t + 1), repeat=3) if sum(map(abs, d)) <= t]
    for z, y, x in itertools.product(range(nz), range(ny), range(nx)):
        if vol[z, y, x] == 0:
            continue
        for dz, dy, dx in offs:
            q = (z + dz, y + dy, x + dx)
            if not (0 <= q[0] < nz and 0 <= q[1] < ny and 0 <= q[2] < nx) or vol[q] == 0:
                out[z, y, x] = vol[z, y, x]
                break
    return out


@pytest.mark.parametrize("t", [1, 2, 3])
@pytest.mark.parametrize("shape,fill", [((5, 6, 7), 0.85), ((7, 4, 9), 0.95), ((1, 6, 6), 0.9), ((8, 8, 8), 0.99)])
def test_matches_city_block_definition(shape, fill, t):
    rng = np.random.default_rng(sum(shape) + t)
    vol = np.where(rng.random(shape) < fill, rng.integers(1, 65536, size=shape), 0).astype(np.uint16)
    assert np.array_equal(HW.hollow(vol, t), _brute(vol, t))


@pytest.mark.parametrize("t", [1, 2, 3, 5])
@pytest.mark.parametrize("shape", [(9, 10, 11), (4, 20, 30), (13, 13, 13)])
def test_solid_box_keeps_its_outer_layers(shape, t):
    """Every voxel non-zero: the erosions leave the inner box of sides n - 2t."""
    vol = np.full(shape, 7, np.uint16)
    inner = np.prod([max(0, n - 2 * t) for n in shape])
    assert HW.kept_count(vol, t) == int(np.prod(shape)) - int(inner)


@pytest.mark.parametrize("t", [1, 2, 3, 4])
def test_octahedral_shell_around_one_empty_voxel(t):
    """A solid cube of side 4t + 3 with its centre voxel zero keeps the outer
    t layers plus the voxels at city-block distance 1..t from the centre:
    (2t + 1)(2t^2 + 2t + 3) / 3 - 1 of them (the octahedral numbers)."""
    n = 4 * t + 3
    vol = np.full((n, n, n), 500, np.uint16)
    c = n // 2
    vol[c, c, c] = 0
    octa = (2 * t + 1) * (2 * t * t + 2 * t + 3) // 3 - 1
    assert HW.kept_count(vol, t) == n ** 3 - (n - 2 * t) ** 3 + octa


def test_grey_values_kept_and_background_stays_zero():
    rng = np.random.default_rng(3)
    vol = np.where(rng.random((12, 14, 16)) < 0.9, rng.integers(1, 65536, size=(12, 14, 16)), 0).astype(np.uint16)
    out = HW.hollow(vol, 2)
    kept = out != 0
    assert np.array_equal(out[kept], vol[kept])
    assert not np.any(out[vol == 0])
    assert out.dtype == vol.dtype and out.shape == vol.shape


def test_monotone_in_thickness_and_complete_at_half_side():
    rng = np.random.default_rng(4)
    shape = (10, 15, 21)
    vol = np.where(rng.random(shape) < 0.97, 1000, 0).astype(np.uint16)
    prev = HW.shell_mask(vol, 1)
    for t in range(2, 6):
        cur = HW.shell_mask(vol, t)
        assert np.all(cur[prev])
        prev = cur
    assert np.array_equal(HW.hollow(vol, 5), vol)          # ceil(10 / 2) = 5


def test_rejects_zero_thickness_and_handles_empty_volume():
    with pytest.raises(ValueError):
        HW.hollow(np.ones((2, 2, 2), np.uint16), 0)
    assert HW.kept_count(np.zeros((3, 4, 5), np.uint16), 2) == 0
