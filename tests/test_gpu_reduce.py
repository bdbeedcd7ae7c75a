"""GPU parity of the reduction steps against the oracle: bit-exact.

Histogram, threshold / keep mask, fused threshold + pyramid, slicemap atlas,
on the small generated volume and on odd, ragged and degenerate shapes.
"""
import numpy as np
import pytest
import torch

from oracle import reduce as O
from paper_2311_15038_amd import synth
from paper_2311_15038_amd import vr

from gpu_util import banner, bits_to_dev, dev, hist_to_dev, to_dev_u16, u16_np, u32_np, u64_np

pytestmark = pytest.mark.gpu

ODD_SHAPES = [(1, 1, 1), (7, 5, 3), (3, 5, 7), (23, 19, 37), (34, 66, 130), (17, 64, 64),
              (129, 257, 33)]


def _rand_vol(shape, seed, lo=0, hi=65536):
    rng = np.random.default_rng(seed)
    return rng.integers(lo, hi, size=shape, dtype=np.uint16)


# ------------------------------------------------------------ histogram
def test_histogram_small_volume(small_volume):
    banner("histogram 128^3")
    v = to_dev_u16(small_volume)
    h = u64_np(vr.vr_histogram(v))
    assert (h == O.histogram(small_volume)).all()
    ht = u64_np(vr.vr_histogram(v, 0, 3))
    assert (ht == O.histogram(small_volume, 0, 3)).all()


@pytest.mark.parametrize("shape", ODD_SHAPES)
def test_histogram_odd_shapes(shape):
    banner(f"histogram {shape}")
    a = _rand_vol(shape, 1)
    v = to_dev_u16(a)
    assert (u64_np(vr.vr_histogram(v)) == O.histogram(a)).all()
    nz = shape[0]
    for z0, nzr in [(0, min(3, nz)), (nz // 2, nz - nz // 2), (nz - 1, 1), (0, 0)]:
        assert (u64_np(vr.vr_histogram(v, z0, nzr)) == O.histogram(a, z0, nzr)).all()


def test_histogram_concentrated_bins_carry():
    # one value everywhere: every wave takes the ballot path and every LDS
    # counter crosses the 0x8000 mark many times
    banner("histogram constant 160^3")
    a = np.full((160, 160, 160), 4242, dtype=np.uint16)
    a[5, 7, 11] = 65535
    a[0, 0, 0] = 0
    h = u64_np(vr.vr_histogram(to_dev_u16(a)))
    assert (h == O.histogram(a)).all()
    # two interleaved values -> neighbouring packed halves carry independently
    b = np.zeros((96, 128, 128), dtype=np.uint16)
    b[..., ::2] = 1000
    b[..., 1::2] = 1001
    assert (u64_np(vr.vr_histogram(to_dev_u16(b))) == O.histogram(b)).all()


@pytest.mark.parametrize("shape,top", [((128, 128, 128), 3), ((7, 5, 3), 3), ((33, 66, 130), 1),
                                       ((5, 9, 11), 5)])
def test_histogram_with_top(shape, top):
    banner(f"histogram with top {shape} top={top}")
    a = _rand_vol(shape, 11, 0, 3000)
    H, Ht = vr.vr_histogram_with_top(to_dev_u16(a), top)
    assert (u64_np(H) == O.histogram(a)).all()
    assert (u64_np(Ht) == O.histogram(a, 0, top)).all()


def test_histogram_rejects_bad_args():
    v = to_dev_u16(_rand_vol((4, 4, 4), 2))
    with pytest.raises(vr.VrError) as e:
        vr.vr_histogram(v, 2, 5)
    assert e.value.code == -3


# ------------------------------------------------------------ threshold
def _select(H, Ht, rule, param):
    res, bits = vr.vr_select_threshold(hist_to_dev(H), None if Ht is None else hist_to_dev(Ht),
                                       rule, param)
    return u32_np(res), u32_np(bits)


def test_valley_and_filter_small_volume(small_volume):
    banner("select valley 128^3")
    H, Ht = O.histogram(small_volume), O.histogram(small_volume, 0, 3)
    res, bits = _select(H, Ht, vr.RULE_VALLEY, 32)
    T = O.valley_threshold(H, 32)
    assert res[0] == T
    assert (bits == O.keep_bits(T, Ht)).all()
    res, bits = _select(H, None, vr.RULE_VALLEY, 32)
    assert res[0] == T and (bits == O.keep_bits(T)).all()
    res, bits = _select(H, Ht, vr.RULE_NONE, 0)
    assert res[0] == 0 and (bits == O.keep_bits(0, Ht)).all()


def _hand_histograms():
    out = []
    H = np.zeros(65536, np.uint64)
    out.append(H.copy())                                # all zero
    H[1000] = 5
    out.append(H.copy())                                # single bin
    H = np.zeros(65536, np.uint64)
    H[100:141] = 1000
    H[500:601] = 10
    out.append(H)
    H = np.zeros(65536, np.uint64)
    H[200] = 50
    H[400] = 50
    out.append(H)
    H = np.zeros(65536, np.uint64)
    H[1000:1065] = 10
    H[1075:1095] = 15
    H[3000:3065] = 10
    out.append(H)
    H = np.zeros(65536, np.uint64)
    H[0], H[65535] = 7, 9                               # extremes
    out.append(H)
    rng = np.random.default_rng(3)
    for _ in range(4):
        c1 = int(rng.integers(200, 5000))
        c2 = c1 + int(rng.integers(2000, 20000))
        H = np.bincount(np.clip(rng.normal(c1, 60, 200000).round().astype(int), 0, 65535),
                        minlength=65536).astype(np.uint64)
        H += np.bincount(np.clip(rng.normal(c2, 300, 20000).round().astype(int), 0, 65535),
                         minlength=65536).astype(np.uint64)
        out.append(H)
    return out


@pytest.mark.parametrize("r", [1, 32, 200])
def test_valley_hand_built(r):
    banner(f"select valley hand-built r={r}")
    for H in _hand_histograms():
        res, bits = _select(H, None, vr.RULE_VALLEY, r)
        T = O.valley_threshold(H, r)
        assert res[0] == T
        assert (bits == O.keep_bits(T)).all()


@pytest.mark.parametrize("shift", [0, 4, 8])
def test_otsu_and_its(small_volume, shift):
    banner(f"select otsu/its shift={shift}")
    hs = [O.histogram(small_volume)] + _hand_histograms()[1:]
    for H in hs:
        Hc = H.reshape(-1, 1 << shift).sum(axis=1)
        res, bits = _select(H, None, vr.RULE_OTSU, shift)
        T = O.otsu_threshold(Hc) << shift
        assert res[0] == T
        assert (bits == O.keep_bits(T)).all()
        res, _ = _select(H, None, vr.RULE_ITS, shift)
        Ti, it = O.its_threshold(Hc)
        assert res[0] == Ti << shift and res[1] == it


def test_select_rejects_bad_rule():
    H = hist_to_dev(np.zeros(65536, np.uint64))
    with pytest.raises(vr.VrError):
        vr.vr_select_threshold(H, None, 7, 0)
    with pytest.raises(vr.VrError):
        vr.vr_select_threshold(H, None, vr.RULE_VALLEY, 0)


# ------------------------------------------------------------ pyramid
def _check_pyramid(a, bits, n_levels):
    v = to_dev_u16(a)
    kb = None if bits is None else bits_to_dev(bits)
    got = vr.vr_threshold_downsample(v, kb, n_levels)
    want = O.pyramid(a, bits, n_levels)
    for k in range(n_levels):
        g = u16_np(got[k])
        assert g.shape == want[k].shape
        assert (g == want[k]).all(), f"level {k + 1} differs at {np.argwhere(g != want[k])[:5]}"


def test_pyramid_small_volume(small_volume):
    banner("pyramid 128^3")
    H, Ht = O.histogram(small_volume), O.histogram(small_volume, 0, 3)
    bits = O.keep_bits(O.valley_threshold(H), Ht)
    _check_pyramid(small_volume, bits, 4)
    _check_pyramid(small_volume, None, 4)
    _check_pyramid(small_volume, bits, 1)


@pytest.mark.parametrize("shape", ODD_SHAPES)
@pytest.mark.parametrize("n_levels", [1, 2, 4])
def test_pyramid_odd_shapes(shape, n_levels):
    banner(f"pyramid {shape} K={n_levels}")
    a = _rand_vol(shape, 4)
    keep = np.random.default_rng(5).random(65536) < 0.7
    _check_pyramid(a, O.pack_bits(keep), n_levels)


def test_pyramid_extreme_values():
    banner("pyramid max values")
    a = np.full((32, 48, 64), 65535, dtype=np.uint16)
    _check_pyramid(a, None, 4)
    a = np.full((31, 47, 65), 65535, dtype=np.uint16)   # ragged: borders darken
    _check_pyramid(a, None, 4)


def test_pyramid_rejects_bad_levels():
    v = to_dev_u16(_rand_vol((8, 8, 8), 6))
    with pytest.raises(vr.VrError) as e:
        vr.vr_threshold_downsample(v, None, 9)
    assert e.value.code == -3


# shapes (nz, ny, nx) whose level-4 grid is ragged, so that the level-5..8 boxes are clipped
DEEP_SHAPES = [(37, 50, 29), (96, 17, 260), (129, 64, 33), (16, 16, 16), (1, 1, 1), (5, 3, 2)]


@pytest.mark.parametrize("shape", DEEP_SHAPES)
@pytest.mark.parametrize("n_levels", [5, 8])
def test_pyramid_eight_levels_and_exact_sums(shape, n_levels):
    """Levels past the fourth are summed from the exact level-4 sums after the
    pass: every level bit-exact against the oracle's own box sums, and every
    exact sum (u64) equal to the oracle's."""
    banner(f"pyramid {shape} K={n_levels} with sums")
    a = _rand_vol(shape, 7)
    keep = np.random.default_rng(8).random(65536) < 0.6
    bits = O.pack_bits(keep)
    v = to_dev_u16(a)
    levels, sums = vr.vr_threshold_downsample(v, bits_to_dev(bits), n_levels, sums=True)
    f = O.apply_keep(a, bits)
    for k in range(1, n_levels + 1):
        S = O.box_sums(f, k)
        assert np.array_equal(sums[k - 1].cpu().numpy(), S), k
        assert np.array_equal(u16_np(levels[k - 1]), O.level_from_sums(S, k)), k
    # without asking for the sums (the binding then passes a level-4 buffer of its own),
    # and the fused levels unchanged by the deeper call
    plain = vr.vr_threshold_downsample(v, bits_to_dev(bits), n_levels)
    four = vr.vr_threshold_downsample(v, bits_to_dev(bits), 4)
    for k in range(n_levels):
        assert torch.equal(plain[k], levels[k]), k
    for k in range(4):
        assert torch.equal(four[k], levels[k]), k


def test_pyramid_atlas_of_a_deep_level():
    banner("atlas of level 6")
    a = _rand_vol((200, 130, 300), 9)
    v = to_dev_u16(a)
    want = O.pyramid(a, None, 6)
    lz, ly, lx = want[5].shape
    tx, ty = 2, 2
    for bits_out in (16, 8):
        atl = torch.full((ty * ly * tx * lx,), 77, dtype=torch.uint16 if bits_out == 16 else torch.uint8,
                         device=v.device)
        got = vr.vr_threshold_downsample(v, None, 6, atlas=(6, tx, ty, bits_out, atl))
        assert np.array_equal(u16_np(got[5]), want[5])
        ref = O.slicemap(want[5], tx, ty, bits_out)
        got_atl = u16_np(atl) if bits_out == 16 else atl.cpu().numpy()
        assert np.array_equal(got_atl.reshape(ref.shape), ref)


# ------------------------------------------------------------ slicemap
@pytest.mark.parametrize("shape,tx,ty", [((64, 64, 64), 8, 8), ((5, 3, 4), 3, 2),
                                          ((7, 2, 9), 2, 5), ((33, 17, 300), 6, 6)])
@pytest.mark.parametrize("bits", [16, 8])
def test_slicemap(shape, tx, ty, bits):
    banner(f"slicemap {shape} {tx}x{ty} {bits}-bit")
    L = _rand_vol(shape, 7)
    got = vr.vr_pack_slicemap(to_dev_u16(L), tx, ty, bits)
    want = O.slicemap(L, tx, ty, bits)
    g = u16_np(got) if bits == 16 else got.cpu().numpy()
    assert g.shape == want.shape and (g == want).all()


@pytest.mark.parametrize("shape,level,tx,ty,bits", [((64, 64, 64), 2, 4, 4, 16), ((34, 66, 130), 1, 5, 4, 16),
                                                     ((37, 23, 19), 2, 3, 4, 8), ((128, 128, 128), 2, 8, 8, 16)])
def test_pyramid_with_atlas(shape, level, tx, ty, bits):
    banner(f"pyramid + atlas {shape} level {level}")
    a = _rand_vol(shape, 12)
    keep = np.random.default_rng(13).random(65536) < 0.8
    bv = O.pack_bits(keep)
    lz, ly, lx = vr.level_shape(shape, level)
    dt = torch.uint16 if bits == 16 else torch.uint8
    atl = torch.full((ty * ly, tx * lx), 77, dtype=torch.int32).to(dt).to(dev())   # stale contents
    got = vr.vr_threshold_downsample(to_dev_u16(a), bits_to_dev(bv), 2, atlas=(level, tx, ty, bits, atl))
    want = O.pyramid(a, bv, 2)
    for k in range(2):
        assert (u16_np(got[k]) == want[k]).all()
    g = u16_np(atl) if bits == 16 else atl.cpu().numpy()
    assert (g == O.slicemap(want[level - 1], tx, ty, bits)).all()


def test_slicemap_rejects_too_few_tiles():
    L = to_dev_u16(_rand_vol((10, 4, 4), 8))
    with pytest.raises(vr.VrError):
        vr.vr_pack_slicemap(L, 3, 3, 16)


# ------------------------------------------------------------ whole reduction
def test_reduction_chain_small_config(small_volume):
    """Histogram -> valley + top-slice filter -> 64^3 level -> 512 x 512 atlas."""
    banner("reduction chain 128^3")
    v = to_dev_u16(small_volume)
    H = vr.vr_histogram(v)
    Ht = vr.vr_histogram(v, 0, 3)
    res, bits = vr.vr_select_threshold(H, Ht, vr.RULE_VALLEY, 32)
    (L1,) = vr.vr_threshold_downsample(v, bits, 1)
    atlas = vr.vr_pack_slicemap(L1, 8, 8, 16)
    Ho, Hto = O.histogram(small_volume), O.histogram(small_volume, 0, 3)
    T = O.valley_threshold(Ho)
    L1o = O.pyramid(small_volume, O.keep_bits(T, Hto), 1)[0]
    assert u32_np(res)[0] == T
    assert (u16_np(L1) == L1o).all()
    assert (u16_np(atlas) == O.slicemap(L1o, 8, 8)).all()


def test_histograms_with_paired_bins_ragged():
    """A volume large enough (>= 2^25 voxels) for the bins to be kept in 32-bit
    pairs during counting, with a ragged shape and uniform values (every bin
    busy): all three histogram calls against the oracle."""
    from oracle import container as K
    shape = (1000, 257, 131)                                # 33.7 M voxels
    banner(f"histogram paired bins {shape}")
    a = _rand_vol(shape, 12)
    assert a.size >= 1 << 25
    v = to_dev_u16(a)
    H = O.histogram(a)
    assert np.array_equal(u64_np(vr.vr_histogram(v)), H)
    assert np.array_equal(u64_np(vr.vr_histogram(v, 100, 900)), O.histogram(a, 100, 900))
    h, ht = vr.vr_histogram_with_top(v, 3)
    assert np.array_equal(u64_np(h), H) and np.array_equal(u64_np(ht), O.histogram(a, 0, 3))
    rec = np.array([1, 70, 120, 100, 96, 1, 1, 1], dtype=np.int32)
    h, ht = vr.vr_histogram_in_disc(v, torch.from_numpy(rec).to(dev()), 3)
    assert np.array_equal(u64_np(h), K.histogram_in_disc(a, rec))
    assert np.array_equal(u64_np(ht), K.histogram_in_disc(a, rec, 0, 3))
