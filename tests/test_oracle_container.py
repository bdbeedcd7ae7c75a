"""Pins of the container-removal oracle (Section III-B) to facts that do not
come from the oracle itself: closed forms of the Sobel operator and of
digital lines, brute force, exact rational arithmetic, the Gauss circle
count, symmetry of the circle under translation and transposition, and the
known geometry of drawn rings and of the generated scene."""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import container as K
from oracle import reduce as O
from paper_2311_15038_amd import synth


def _ring(n, cx, cy, r0, w, inside=1000, wall=7000, outside=1000):
    X = np.arange(n)[None, :] - cx
    Y = np.arange(n)[:, None] - cy
    d2 = X * X + Y * Y
    s = np.full((n, n), outside, np.int64)
    s[d2 < r0 * r0] = inside
    s[(d2 >= r0 * r0) & (d2 <= (r0 + w) ** 2)] = wall
    return s.astype(np.uint16)


def test_sobel_of_a_plane_is_eight_times_its_slope():
    y, x = np.mgrid[0:9, 0:11]
    s = 3 * x + 5 * y + 100
    gx, gy = K.sobel(s)
    assert (gx[1:-1, 1:-1] == 24).all() and (gy[1:-1, 1:-1] == 40).all()
    assert (gx[0] == 0).all() and (gx[:, -1] == 0).all() and (gy[-1] == 0).all()


def test_sobel_brute_force():
    rng = np.random.default_rng(0)
    s = rng.integers(0, 65536, size=(7, 6))
    gx, gy = K.sobel(s)
    for y in range(1, 6):
        for x in range(1, 5):
            p = lambda dy, dx: int(s[y + dy, x + dx])  # noqa: E731
            ex = (p(-1, 1) + 2 * p(0, 1) + p(1, 1)) - (p(-1, -1) + 2 * p(0, -1) + p(1, -1))
            ey = (p(1, -1) + 2 * p(1, 0) + p(1, 1)) - (p(-1, -1) + 2 * p(-1, 0) + p(-1, 1))
            assert gx[y, x] == ex and gy[y, x] == ey


def test_edge_threshold_is_relative_to_the_largest_gradient():
    s = np.zeros((8, 8), np.int64)
    s[:, 4:] = 100          # step: |gx| = 400 on columns 3 and 4
    s[6, 1] = 20            # a small bump: gradient magnitude <= 40 < 400 / 4
    x, y, gx, gy = K.edge_pixels(s, 4)
    assert set(x.tolist()) == {3, 4} and (np.abs(gx) == 400).all()
    x2, *_ = K.edge_pixels(s, 8)           # threshold 400 / 16 = 25 admits the bump
    assert x2.size > x.size


def test_digital_line_closed_forms():
    x, y = np.array([50]), np.array([40])
    for k in range(1, 6):
        assert K.line_cells(x, y, np.array([5]), np.array([0]), k) == (50 - k, 40)
        assert K.line_cells(x, y, np.array([0]), np.array([-7]), k) == (50, 40 + k)
        assert K.line_cells(x, y, np.array([4]), np.array([4]), k) == (50 - k, 40 - k)
        assert K.line_cells(x, y, np.array([-3]), np.array([3]), k) == (50 + k, 40 - k)
    # slope 1/2 along x: minor offsets round(k / 2) with halves up = 1, 1, 2, 2, 3
    got = [K.line_cells(x, y, np.array([2]), np.array([1]), k)[1][0] for k in range(1, 6)]
    assert got == [39, 39, 38, 38, 37]


def test_digital_line_is_the_nearest_cell_exactly():
    """Minor offset = the integer nearest to k gmin / gmaj (halves up), exact rationals."""
    rng = np.random.default_rng(1)
    g = rng.integers(-262140, 262141, size=(4000, 2))
    g = g[(g != 0).any(axis=1)]
    k = rng.integers(1, 4097, size=g.shape[0])
    cx, cy = K.line_cells(np.zeros_like(k), np.zeros_like(k), g[:, 0], g[:, 1], k)
    for i in range(g.shape[0]):
        a, b = abs(int(g[i, 0])), abs(int(g[i, 1]))
        gmaj, gmin = max(a, b), min(a, b)
        q = Fraction(int(k[i]) * gmin, gmaj)
        j = math.floor(q + Fraction(1, 2))
        ox, oy = (int(k[i]), j) if a >= b else (j, int(k[i]))
        assert -cx[i] == ox * int(np.sign(g[i, 0])) and -cy[i] == oy * int(np.sign(g[i, 1]))


def test_step_range_is_the_euclidean_distance():
    rng = np.random.default_rng(2)
    g = rng.integers(-262140, 262141, size=(3000, 2))
    g = g[(g != 0).any(axis=1)]
    k = rng.integers(1, 4097, size=g.shape[0])
    r_min, r_max = 500, 2000
    ok = K.step_in_range(g[:, 0], g[:, 1], k, r_min, r_max)
    for i in range(g.shape[0]):
        gmaj = max(abs(int(g[i, 0])), abs(int(g[i, 1])))
        d = int(k[i]) * math.hypot(int(g[i, 0]), int(g[i, 1])) / gmaj
        if abs(d - r_min) < 1e-6 or abs(d - r_max) < 1e-6:
            continue
        assert bool(ok[i]) == (r_min <= d <= r_max)


def test_round_sqrt_exact():
    D = np.arange(0, 200000)
    d = K.round_sqrt(D)
    ref = np.array([math.isqrt(4 * int(v)) for v in D])      # floor(2 sqrt(D))
    assert np.array_equal(d, (ref + 1) // 2)                  # floor(sqrt(D) + 1/2)


def test_accumulator_of_a_straight_edge_brute_force():
    n = 40
    s = np.zeros((n, n), np.int64)
    s[:, 25:] = 500                               # rising to the right: lines run to -x
    r_min, r_max = 3, 12
    acc, (x, y, gx, gy) = K.accumulator(s, r_min, r_max, 4)
    ref = np.zeros((n, n), np.int64)
    for xe, ye, a, b in zip(x, y, gx, gy):
        assert b == 0 and a > 0
        for r in range(r_min, r_max + 1):
            if xe - r >= 0:
                ref[ye, xe - r] += 1
    assert np.array_equal(acc, ref)


def test_box_sums_brute_force():
    rng = np.random.default_rng(3)
    a = rng.integers(0, 9, size=(13, 17))
    for w in (1, 2, 5):
        B = K.box_sums(a, w)
        for y in range(13):
            for x in range(17):
                assert B[y, x] == a[max(0, y - w):y + w + 1, max(0, x - w):x + w + 1].sum()


@pytest.mark.parametrize("cx,cy,r0", [(64, 62, 50), (70, 57, 40), (60, 66, 30)])
def test_clean_ring_centre_and_radius(cx, cy, r0):
    s = _ring(128, cx, cy, r0, 4)
    rec = K.find_container(s, 16, 64, 4, 2)
    assert rec[0] == 1 and (rec[1], rec[2]) == (cx, cy)
    assert abs(rec[3] - r0) <= 1 and rec[4] == rec[3] - 2


def test_translation_moves_the_centre():
    rng = np.random.default_rng(4)
    base = _ring(128, 60, 61, 44, 4).astype(np.int64) + rng.integers(0, 200, size=(128, 128))
    r0 = K.find_container(base, 16, 64, 4, 2)
    sh = np.roll(np.roll(base, 7, axis=1), -5, axis=0)
    r1 = K.find_container(sh, 16, 64, 4, 2)
    assert (r1[1] - r0[1], r1[2] - r0[2]) == (7, -5) and r1[3] == r0[3]


def test_transpose_swaps_the_centre():
    s = synth.to_numpy_u16(synth.make_volume(synth.VolumeSpec(128, 128, 4, seed=5, container=synth.CONTAINER_RING)))[0]
    a = K.find_container(s, 16, 64, 4, 2)
    b = K.find_container(np.ascontiguousarray(s.T), 16, 64, 4, 2)
    assert (b[1], b[2]) == (a[2], a[1]) and b[3] == a[3]


def test_the_container_wins_over_a_bright_specimen():
    s = _ring(128, 64, 64, 55, 4).astype(np.int64)
    Y, X = np.mgrid[0:128, 0:128]
    s[(X - 52) ** 2 + (Y - 70) ** 2 <= 18 ** 2] = 9000     # bright disc inside the container
    rec = K.find_container(s, 10, 64, 4, 2)
    assert (rec[1], rec[2]) == (64, 64) and abs(rec[3] - 55) <= 1


def test_constant_slice_finds_nothing():
    s = np.full((32, 48), 1234, np.uint16)
    rec = K.find_container(s, 4, 16, 4, 2)
    assert rec.tolist() == [0] * 8
    vol = np.full((3, 32, 48), 7, np.uint16)
    assert K.disc_mask(48, 32, rec).all()
    assert np.array_equal(K.histogram_in_disc(vol, rec), O.histogram(vol))


def _gauss_circle(R):
    return 1 + 4 * R + 4 * sum(math.isqrt(R * R - i * i) for i in range(1, R + 1))


@pytest.mark.parametrize("R", [0, 1, 5, 17, 30])
def test_disc_count_is_the_gauss_circle_number(R):
    rec = np.array([1, 31, 33, R + 2, R, 1, 1, 1])
    m = K.disc_mask(64, 70, rec)
    assert int(m.sum()) == _gauss_circle(R)
    vol = np.random.default_rng(R).integers(0, 65536, size=(3, 70, 64)).astype(np.uint16)
    assert int(K.histogram_in_disc(vol, rec).sum()) == 3 * _gauss_circle(R)
    assert int(K.histogram_in_disc(vol, rec, 1, 1).sum()) == _gauss_circle(R)


def test_removal_zeroes_exactly_the_outside():
    rng = np.random.default_rng(6)
    vol = rng.integers(1, 65536, size=(4, 50, 60)).astype(np.uint16)
    rec = np.array([1, 25, 22, 20, 18, 1, 1, 1])
    out = K.remove_container(vol, rec)
    m = K.disc_mask(60, 50, rec)
    assert (out[:, ~m] == 0).all() and np.array_equal(out[:, m], vol[:, m])
    H = O.histogram(out)
    Hd = K.histogram_in_disc(vol, rec)
    n_out = 4 * int((~m).sum())
    assert int(H[0]) == n_out and np.array_equal(H[1:], Hd[1:])


@pytest.fixture(scope="module")
def contained():
    v = synth.to_numpy_u16(synth.make_volume(synth.SMALL_CONTAINED))
    lab = synth.make_labels(synth.SMALL_CONTAINED).numpy()
    return v, lab, K.find_container(v[0], 16, 64, 4, 2)


def test_generated_container_is_found(contained):
    v, lab, rec = contained
    cx, cy, r0, _ = synth.CONTAINER_RING          # base frame = voxels at 128^3
    assert rec[0] == 1
    assert abs(rec[1] - (cx - 0.5)) <= 1.5 and abs(rec[2] - (cy - 0.5)) <= 1.5
    assert abs(rec[3] - r0) <= 1
    m = K.disc_mask(128, 128, rec)
    assert not ((lab == synth.CONTAINER) & m[None]).any()                 # no wall kept
    assert not ((lab > 0) & (lab != synth.CONTAINER) & ~m[None]).any()   # no specimen lost


def test_removal_keeps_the_specimen_that_the_top_filter_loses(contained):
    """The top slices show the wall, so without removal the top-slice filter
    drops the wall's grey values, which the outer shell shares; with removal
    the top-slice histogram holds air only (Section III-B, III-D)."""
    v, lab, rec = contained
    m = K.disc_mask(128, 128, rec)
    H, Ht = O.histogram(v), O.histogram(v, 0, 3)
    Hd, Htd = K.histogram_in_disc(v, rec), K.histogram_in_disc(v, rec, 0, 3)
    assert int(np.nonzero(Htd)[0].max()) < 2000 < int(np.nonzero(Ht)[0].max())
    keep = O.unpack_bits(O.keep_bits(O.valley_threshold(H), Ht))
    keep_d = O.unpack_bits(O.keep_bits(O.valley_threshold(Hd), Htd))
    outer = lab == synth.OUTER
    assert keep_d[v[outer]].all() and keep[v[outer]].mean() < 0.95
    assert not (keep_d[v] & m[None])[lab == synth.CONTAINER].any()
