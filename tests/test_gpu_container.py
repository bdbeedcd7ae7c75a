"""GPU parity of container removal (Section III-B) against the oracle, exact:
the circle record of the Hough search, the histograms of the voxels inside
the kept disc, the removal in place, and the pyramid with the disc applied,
on generated slices and volumes, ragged and degenerate shapes, discs that
cross the slice's border and circles that were not found."""
import numpy as np
import pytest
import torch

from oracle import container as K
from oracle import reduce as O
from paper_2311_15038_amd import pipeline as P
from paper_2311_15038_amd import synth
from paper_2311_15038_amd import vr

from gpu_util import banner, bits_to_dev, dev, hist_to_dev, to_dev_u16, u16_np, u64_np

pytestmark = pytest.mark.gpu


def _ring(nx, ny, cx, cy, r0, w):
    X = np.arange(nx)[None, :] - cx
    Y = np.arange(ny)[:, None] - cy
    d2 = X * X + Y * Y
    s = np.full((ny, nx), 1000, np.uint16)
    s[(d2 >= r0 * r0) & (d2 <= (r0 + w) ** 2)] = 7000
    return s


def _scene_slice(nx, ny, seed, noise="gauss"):
    spec = synth.VolumeSpec(nx, ny, 4, seed=seed, noise=noise, container=synth.CONTAINER_RING)
    return synth.to_numpy_u16(synth.make_volume(spec))[0]


def _slices():
    rng = np.random.default_rng(5)
    small = synth.to_numpy_u16(synth.make_volume(synth.SMALL_CONTAINED))[0]
    return {
        "small_contained": (small, 16, 64, 4, 2),
        "ragged_150x97": (_scene_slice(150, 97, 7), 12, 48, 4, 2),
        "clean_ring": (_ring(128, 128, 64, 62, 50, 4), 16, 64, 4, 2),
        "edge_shift_0_margin_99": (small, 16, 64, 0, 99),
        "constant": (np.full((80, 100), 1234, np.uint16), 10, 40, 4, 2),
        "uniform_noise": (rng.integers(0, 65536, size=(80, 64)).astype(np.uint16), 8, 32, 4, 2),
        "three_by_three": (rng.integers(0, 65536, size=(3, 3)).astype(np.uint16), 1, 2, 4, 0),
        "huge_window": (_ring(64, 64, 30, 33, 20, 3), 1, 4096, 4, 2),
        "step_edge": (np.repeat(np.where(np.arange(90) < 50, 100, 900)[None, :], 70, axis=0).astype(np.uint16),
                      5, 30, 4, 1),
    }


SLICES = _slices()


@pytest.mark.parametrize("name", list(SLICES))
def test_circle_record_matches_oracle(name):
    s, r0, r1, sh, m = SLICES[name]
    banner(f"container: find on {name} {s.shape}")
    got = vr.vr_find_container(to_dev_u16(s), r0, r1, sh, m).cpu().numpy()
    ref = K.find_container(s, r0, r1, sh, m)
    assert got.tolist() == ref.tolist(), (got, ref)


def test_generated_container_found_on_device():
    s = SLICES["small_contained"][0]
    rec = vr.vr_find_container(to_dev_u16(s), 16, 64).cpu().numpy()
    assert rec[0] == 1 and abs(rec[3] - 60) <= 1
    assert abs(rec[1] - 64.1) <= 1.5 and abs(rec[2] - 62.8) <= 1.5


def test_workspace_reuse_gives_the_same_record():
    """A second search in the same workspace clears what the first left there."""
    banner("container: workspace reuse")
    a, b = SLICES["ragged_150x97"][0], _scene_slice(150, 97, 8)
    need = vr.vr_container_workspace_size(150, 97, 48)
    work = torch.empty(need, dtype=torch.uint8, device=dev())
    r1 = vr.vr_find_container(to_dev_u16(a), 12, 48, work=work).cpu().numpy()
    r2 = vr.vr_find_container(to_dev_u16(b), 12, 48, work=work).cpu().numpy()
    assert r1.tolist() == K.find_container(a, 12, 48).tolist()
    assert r2.tolist() == K.find_container(b, 12, 48).tolist()


# records chosen by hand: inside, crossing the border, a single column, not found
RECORDS = {
    "inside": [1, 60, 50, 40, 37, 1, 1, 1],
    "crosses_border": [1, 10, 90, 32, 30, 1, 1, 1],
    "radius_zero": [1, 33, 20, 2, 0, 1, 1, 1],
    "outside_slice": [1, 500, 500, 12, 10, 1, 1, 1],
    "not_found": [0, 0, 0, 0, 0, 0, 0, 0],
}
SHAPES = [(45, 97, 131), (16, 128, 256), (5, 3, 7), (7, 61, 24), (3, 1, 8)]


def _rand_vol(shape, seed):
    return np.random.default_rng(seed).integers(0, 65536, size=shape, dtype=np.uint16)


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("rname", list(RECORDS))
def test_histograms_in_disc(shape, rname):
    banner(f"container: histograms in disc {shape} {rname}")
    a = _rand_vol(shape, 2)
    rec = np.array(RECORDS[rname], dtype=np.int32)
    top = min(3, shape[0])
    H, Ht = vr.vr_histogram_in_disc(to_dev_u16(a), torch.from_numpy(rec).to(dev()), top)
    assert np.array_equal(u64_np(H), K.histogram_in_disc(a, rec))
    assert np.array_equal(u64_np(Ht), K.histogram_in_disc(a, rec, 0, top))
    H2, none = vr.vr_histogram_in_disc(to_dev_u16(a), torch.from_numpy(rec).to(dev()), 0)
    assert none is None and np.array_equal(u64_np(H2), K.histogram_in_disc(a, rec))


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("rname", list(RECORDS))
def test_removal_in_place(shape, rname):
    banner(f"container: removal {shape} {rname}")
    a = _rand_vol(shape, 3)
    rec = np.array(RECORDS[rname], dtype=np.int32)
    v = to_dev_u16(a)
    vr.vr_remove_container(v, torch.from_numpy(rec).to(dev()))
    assert np.array_equal(u16_np(v), K.remove_container(a, rec))


def _keep_variants(a, rec):
    H, Ht = K.histogram_in_disc(a, rec), K.histogram_in_disc(a, rec, 0, min(3, a.shape[0]))
    T = O.valley_threshold(H)
    return {"all": None, "interval": O.keep_bits(T), "lookup": O.keep_bits(T, Ht)}


@pytest.mark.parametrize("shape", [(45, 97, 131), (32, 64, 512), (9, 17, 8)])
@pytest.mark.parametrize("rname", ["inside", "crosses_border", "not_found"])
def test_pyramid_in_disc(shape, rname):
    a = _rand_vol(shape, 4)
    rec = np.array(RECORDS[rname], dtype=np.int32)
    cleaned = K.remove_container(a, rec)
    v, c = to_dev_u16(a), torch.from_numpy(rec).to(dev())
    for kname, bits in _keep_variants(a, rec).items():
        banner(f"container: pyramid in disc {shape} {rname} keep={kname}")
        kb = None if bits is None else bits_to_dev(bits)
        ref = O.pyramid(cleaned, bits, 4)
        lz, ly, lx = vr.level_shape(shape, 2)
        tx, ty = P.atlas_tiles(lz)
        atlas = torch.empty((ty * ly, tx * lx), dtype=torch.uint16, device=dev())
        got = vr.vr_threshold_downsample(v, kb, 4, atlas=(2, tx, ty, 16, atlas), circle=c)
        for k in range(4):
            assert np.array_equal(u16_np(got[k]), ref[k]), (kname, k + 1)
        assert np.array_equal(u16_np(atlas), O.slicemap(ref[1], tx, ty, 16))
    assert np.array_equal(u16_np(v), a)                  # the input is left as it was


@pytest.mark.parametrize("shape", [(45, 97, 131), (40, 64, 512)])
def test_pyramid_in_disc_eight_levels_with_sums(shape):
    """The in-disc pass with levels past the fourth (summed from its exact level-4
    sums) and every level's exact sums, against the oracle on the container-removed
    volume."""
    a = _rand_vol(shape, 5)
    rec = np.array(RECORDS["crosses_border"], dtype=np.int32)
    cleaned = K.remove_container(a, rec)
    bits = _keep_variants(a, rec)["lookup"]
    banner(f"container: 8-level pyramid in disc {shape}")
    levels, sums = vr.vr_threshold_downsample(to_dev_u16(a), bits_to_dev(bits), 8,
                                              circle=torch.from_numpy(rec).to(dev()), sums=True)
    f = O.apply_keep(cleaned, bits)
    for k in range(1, 9):
        S = O.box_sums(f, k)
        assert np.array_equal(sums[k - 1].cpu().numpy(), S), k
        assert np.array_equal(u16_np(levels[k - 1]), O.level_from_sums(S, k)), k


def test_pipeline_with_container_matches_oracle():
    banner("container: preview pipeline on the small contained scene")
    a = synth.to_numpy_u16(synth.make_volume(synth.SMALL_CONTAINED))
    cfg = P.PreviewConfig(n_views=2, width=128, height=128, container=True)
    pipe = P.PreviewPipeline(a.shape, cfg, device=dev())
    v = to_dev_u16(a)
    pipe.step(v)
    torch.cuda.synchronize()
    rec = K.find_container(a[0], 16, 64, 4, 2)
    assert pipe.circle.cpu().numpy().tolist() == rec.tolist()
    H, Ht = K.histogram_in_disc(a, rec), K.histogram_in_disc(a, rec, 0, 3)
    assert np.array_equal(u64_np(pipe.hist), H) and np.array_equal(u64_np(pipe.hist_top), Ht)
    T = O.valley_threshold(H)
    assert int(pipe.result[0].item()) == T
    ref = O.pyramid(K.remove_container(a, rec), O.keep_bits(T, Ht), 4)
    for k in range(4):
        assert np.array_equal(u16_np(pipe.levels[k]), ref[k])
    # a second step on the untouched volume gives the same circle and levels
    pipe.step(v)
    torch.cuda.synchronize()
    assert pipe.circle.cpu().numpy().tolist() == rec.tolist()
    assert np.array_equal(u16_np(pipe.levels[0]), ref[0])


def test_selection_on_disc_histograms():
    """Otsu and ITS on the in-disc histogram of the contained scene (Section III-B's
    point: the container shifts the histogram these rules read)."""
    a = synth.to_numpy_u16(synth.make_volume(synth.SMALL_CONTAINED))
    rec = K.find_container(a[0], 16, 64, 4, 2)
    H = K.histogram_in_disc(a, rec)
    for shift in (8, 0):
        Hc = H.reshape(-1, 1 << shift).sum(axis=1)
        res, _ = vr.vr_select_threshold(hist_to_dev(H), None, vr.RULE_OTSU, shift)
        assert int(res[0].item()) == O.otsu_threshold(Hc) << shift
        res, _ = vr.vr_select_threshold(hist_to_dev(H), None, vr.RULE_ITS, shift)
        Ti, it = O.its_threshold(Hc)
        assert int(res[0].item()) == Ti << shift and int(res[1].item()) == it
