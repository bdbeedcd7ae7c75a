"""Pins for the reduction oracle against facts the paper and the mathematics fix.

Each test checks the oracle against something other than itself: brute-force
loops on tiny inputs, invariants, hand-derived values, or an independent
formulation (Eq. 1's within-class variance for Otsu, the fixed-point property
for ITS).
"""
from fractions import Fraction

import numpy as np
import pytest

from oracle import reduce as O


def _tiny(seed, shape=(7, 5, 3)):
    rng = np.random.default_rng(seed)
    # few distinct values so bins repeat, plus extremes
    v = rng.choice(np.array([0, 1, 2, 7, 1000, 32768, 65535], dtype=np.uint16), size=shape)
    return v


# ------------------------------------------------------------ histogram
@pytest.mark.parametrize("z0,nzr", [(0, 7), (0, 3), (2, 4), (6, 1), (3, 0)])
def test_histogram_brute_force(z0, nzr):
    v = _tiny(1)
    H = O.histogram(v, z0, nzr)
    ref = {}
    for z in range(z0, z0 + nzr):
        for y in range(v.shape[1]):
            for x in range(v.shape[2]):
                ref[int(v[z, y, x])] = ref.get(int(v[z, y, x]), 0) + 1
    assert H.dtype == np.uint64 and H.shape == (65536,)
    for b in range(65536):
        assert H[b] == ref.get(b, 0)


def test_histogram_sums_to_voxel_count(small_volume):
    nz, ny, nx = small_volume.shape
    assert int(O.histogram(small_volume).sum()) == nx * ny * nz
    assert int(O.histogram(small_volume, 0, 3).sum()) == nx * ny * 3


# ------------------------------------------------------------ valley rule
def test_smoothed_brute_force():
    rng = np.random.default_rng(2)
    H = np.zeros(65536, dtype=np.uint64)
    idx = rng.integers(0, 65536, size=500)
    H[idx] = rng.integers(1, 1000, size=500).astype(np.uint64)
    H[0], H[65535] = 5, 7
    S = O.smoothed(H, 32)
    for b in [0, 1, 31, 32, 33, 1000, 40000, 65502, 65503, 65534, 65535]:
        ref = sum(int(H[k]) for k in range(b - 32, b + 33) if 0 <= k < 65536)
        assert int(S[b]) == ref


def test_valley_hand_built_gap():
    # air block on bins 100..140, empty gap, object on 500..600
    H = np.zeros(65536, dtype=np.uint64)
    H[100:141] = 1000
    H[500:601] = 10
    # S > 0 up to b = 140 + 32 = 172, S = 0 on [173, 467], S rises at 468:
    # b* = 467 and its plateau starts at 173.
    assert O.valley_threshold(H, 32) == 173


def test_valley_ties_and_degenerate():
    H = np.zeros(65536, dtype=np.uint64)
    assert O.valley_threshold(H) == 65535            # all zero: no valley
    H[1000] = 5                                       # one bin: S flat then 0, never rises
    assert O.valley_threshold(H) == 65535
    H2 = np.zeros(65536, dtype=np.uint64)
    H2[200] = 50
    H2[400] = 50                                      # equal peaks -> the lower one is p
    # S = 50 on [168, 232], 0 on [233, 367], rises at 368 -> T = 233
    assert O.valley_threshold(H2) == 233
    # a dip that stays above half the peak is not a valley
    H3 = np.zeros(65536, dtype=np.uint64)
    H3[1000:1065] = 10                                # S peaks at 650 on b = 1032
    H3[1075:1095] = 15                                # shoulder: S dips to 550 at 1042, rises
    H3[3000:3065] = 10
    S3 = O.smoothed(H3, 32).astype(np.int64)
    assert S3[1042] == 550 and S3[1043] > S3[1042]    # the shallow dip exists (550 > 650/2)
    # S > 0 up to the shoulder's last bin 1094 + 32, S = 0 on [1127, 2967], rises at 2968
    assert O.valley_threshold(H3) == 1127


def test_valley_properties_random():
    rng = np.random.default_rng(3)
    for trial in range(20):
        H = np.zeros(65536, dtype=np.uint64)
        c1 = int(rng.integers(200, 5000))
        c2 = c1 + int(rng.integers(2000, 20000))
        H += np.bincount(np.clip(rng.normal(c1, 60, 200000).round().astype(int), 0, 65535),
                         minlength=65536).astype(np.uint64)
        H += np.bincount(np.clip(rng.normal(c2, 300, 20000).round().astype(int), 0, 65535),
                         minlength=65536).astype(np.uint64)
        S = O.smoothed(H, 32).astype(np.int64)
        T = O.valley_threshold(H, 32)
        p = int(np.argmax(S))
        assert S[p] == S.max() and (S[:p] < S[p]).all()
        assert p < T < 65535
        bstar = T
        while S[bstar + 1] == S[T]:
            bstar += 1
        assert S[bstar + 1] > S[bstar]
        assert 2 * S[bstar] <= S[p]
        # no earlier bin past half height where S rises
        half = [b for b in range(p + 1, bstar) if 2 * S[b] <= S[p]]
        assert all(S[b + 1] <= S[b] for b in half)
        assert T == p + 1 or S[T - 1] > S[T]
        assert c1 + 2 * 60 < T < c2 - 3 * 300


def test_valley_separates_classes_on_generated_volume(small_volume):
    T = O.valley_threshold(O.histogram(small_volume))
    assert 1000 + 3 * 40 < T < 8000 - 3 * 300


# ------------------------------------------------------------ Otsu / ITS
def _eq1_argmin(H):
    """Eq. 1: minimise the within-class variance w0 s0^2 + w1 s1^2 (exact rationals)."""
    B = len(H)
    N = sum(int(h) for h in H)
    best, bestT = None, None
    for T in range(1, B):
        a = [(b, int(H[b])) for b in range(T) if H[b]]
        c = [(b, int(H[b])) for b in range(T, B) if H[b]]
        na, nc = sum(h for _, h in a), sum(h for _, h in c)
        if na == 0 or nc == 0:
            continue
        ma = Fraction(sum(b * h for b, h in a), na)
        mc = Fraction(sum(b * h for b, h in c), nc)
        va = sum(h * (b - ma) ** 2 for b, h in a) / na
        vc = sum(h * (b - mc) ** 2 for b, h in c) / nc
        w = Fraction(na, N) * va + Fraction(nc, N) * vc
        if best is None or w < best:
            best, bestT = w, T
    return bestT


@pytest.mark.parametrize("seed", range(6))
def test_otsu_matches_eq1_within_class_minimum(seed):
    rng = np.random.default_rng(100 + seed)
    B = 48
    H = np.zeros(B, dtype=np.uint64)
    H[:] = rng.integers(0, 50, size=B)
    H[rng.integers(0, B, size=3)] += rng.integers(100, 400, size=3).astype(np.uint64)
    assert O.otsu_threshold(H) == _eq1_argmin(H)


def test_otsu_two_point_masses_lowest_tie():
    H = np.zeros(256, dtype=np.uint64)
    H[40], H[200] = 1000, 300
    assert O.otsu_threshold(H) == 41                  # every T in (40, 200] ties


def test_its_symmetric_masses():
    H = np.zeros(256, dtype=np.uint64)
    H[50], H[150] = 10, 10
    T, it = O.its_threshold(H)
    assert T == 100 and it <= 3


@pytest.mark.parametrize("seed", range(5))
def test_its_fixed_point(seed):
    rng = np.random.default_rng(200 + seed)
    H = np.zeros(256, dtype=np.uint64)
    H += np.bincount(np.clip(rng.normal(60, 15, 5000).astype(int), 0, 255), minlength=256).astype(np.uint64)
    H += np.bincount(np.clip(rng.normal(170, 20, 3000).astype(int), 0, 255), minlength=256).astype(np.uint64)
    T, it = O.its_threshold(H)
    b = np.arange(256)
    m1 = Fraction(int((b[:T] * H[:T]).sum()), int(H[:T].sum()))
    m2 = Fraction(int((b[T:] * H[T:]).sum()), int(H[T:].sum()))
    assert T == int((m1 + m2) / 2)                    # floor of the exact midpoint
    assert it < 20


# ------------------------------------------------------------ keep mask
def test_keep_bit_order():
    keep = np.zeros(65536, dtype=bool)
    keep[[0, 33, 65535]] = True
    bits = O.pack_bits(keep)
    assert bits.dtype == np.uint32 and bits.shape == (2048,)
    assert bits[0] == 1 and bits[1] == 2 and bits[2047] == 1 << 31
    assert int(np.count_nonzero(bits)) == 3
    assert (O.unpack_bits(bits) == keep).all()


def test_keep_bits_semantics():
    Ht = np.zeros(65536, dtype=np.uint64)
    Ht[[5, 900, 901]] = 3
    bits = O.keep_bits(100, Ht)
    keep = O.unpack_bits(bits)
    for b in [0, 5, 99, 100, 899, 900, 901, 902, 65535]:
        assert keep[b] == (b >= 100 and b not in (5, 900, 901))


# ------------------------------------------------------------ pyramid
@pytest.mark.parametrize("k", [1, 2, 3])
def test_box_sums_brute_force(k):
    v = _tiny(4, (7, 5, 3))
    S = O.box_sums(v.astype(np.int64), k)
    d = 1 << k
    nz, ny, nx = v.shape
    mz, my, mx = -(-nz // d), -(-ny // d), -(-nx // d)
    assert S.shape == (mz, my, mx)
    for z in range(mz):
        for y in range(my):
            for x in range(mx):
                ref = 0
                for zz in range(z * d, z * d + d):
                    for yy in range(y * d, y * d + d):
                        for xx in range(x * d, x * d + d):
                            if zz < nz and yy < ny and xx < nx:
                                ref += int(v[zz, yy, xx])
                assert S[z, y, x] == ref


def test_pyramid_mass_conservation(small_volume):
    T = O.valley_threshold(O.histogram(small_volume))
    f = O.apply_keep(small_volume, O.keep_bits(T))
    tot = int(f.astype(np.int64).sum())
    for k in range(1, 5):
        assert int(O.box_sums(f, k).sum()) == tot


def test_pyramid_constant_and_rounding():
    v = np.full((16, 16, 16), 12345, dtype=np.uint16)
    for k, L in enumerate(O.pyramid(v, None, 4), start=1):
        assert L.shape == (16 >> k,) * 3 and (L == 12345).all()
    # round half up from exact sums
    assert O.level_from_sums(np.array([4, 3, 11, 12]), 1).tolist() == [1, 0, 1, 2]
    assert O.level_from_sums(np.array([32, 31]), 2).tolist() == [1, 0]
    assert O.level_from_sums(np.array([8 * 65535]), 1).tolist() == [65535]


def test_pyramid_levels_not_chained():
    # a 4x4x4 block whose level-1 means each round up: chaining would double-round
    v = np.zeros((4, 4, 4), dtype=np.uint16)
    v[::2, ::2, ::2] = 4                 # each 2-cube sums to 4 -> L1 = 1 (4/8 rounds up)
    L1, L2 = O.pyramid(v, None, 2)
    assert (L1 == 1).all()
    assert L2[0, 0, 0] == (32 + 32) >> 6   # exact: 8 * 4 = 32 over 64 voxels -> 1 (half up)
    v[0, 0, 0] = 3                       # S2 = 31 -> 0, although L1 chaining would give 1
    assert O.pyramid(v, None, 2)[1][0, 0, 0] == 0


def test_box_sum_at_matches(small_volume):
    bits = O.keep_bits(O.valley_threshold(O.histogram(small_volume)))
    f = O.apply_keep(small_volume, bits)
    rng = np.random.default_rng(5)
    for k in (1, 3):
        S = O.box_sums(f, k)
        pos = [tuple(int(rng.integers(0, n)) for n in S.shape) for _ in range(20)]
        assert (O.box_sum_at(small_volume, bits, k, pos) == np.array([S[p] for p in pos])).all()


# ------------------------------------------------------------ slicemap
@pytest.mark.parametrize("shape,tx,ty", [((5, 3, 4), 3, 2), ((8, 8, 8), 4, 2), ((7, 2, 9), 2, 5)])
def test_slicemap_brute_force(shape, tx, ty):
    rng = np.random.default_rng(6)
    L = rng.integers(0, 65536, size=shape).astype(np.uint16)
    A = O.slicemap(L, tx, ty)
    nz, ny, nx = shape
    assert A.shape == (ty * ny, tx * nx)
    for Y in range(A.shape[0]):
        for X in range(A.shape[1]):
            z = (Y // ny) * tx + X // nx
            ref = L[z, Y % ny, X % nx] if z < nz else 0
            assert A[Y, X] == ref


def test_slicemap_8bit():
    L = np.array([0, 127, 128, 383, 384, 65151, 65152, 65535], dtype=np.uint16).reshape(8, 1, 1)
    A = O.slicemap(L, 8, 1, out_bits=8)
    assert A.dtype == np.uint8
    assert A.ravel().tolist() == [0, 0, 1, 1, 2, 254, 255, 255]
