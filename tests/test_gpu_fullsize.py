"""Full-size parity: the 1024^3 volume through the step the benchmark times
(histograms, selection, fused 4-level pyramid with the 256^3 -> 4096^2 atlas,
bricked 512^3 level, 36 x 512^2 turntable frames with empty-space skipping).

Checked against the oracle: both histograms in full; the threshold and keep
mask; every level on sampled 16-slice slabs (box sums never cross them) plus
level 1 in full (built slab by slab); the atlas as the slicemap of level 2;
every pixel of the 36 rendered frames and the step's sample count against
the FP64 oracle's render of its own level 1."""
import numpy as np
import pytest
import torch

from oracle import reduce as O
from oracle import render as R
from paper_2311_15038_amd import pipeline as P
from paper_2311_15038_amd import synth

from gpu_util import banner, dev, u16_np, u32_np, u64_np

pytestmark = pytest.mark.gpu

SLAB = 16                       # 2^4 slices: a slab holds whole boxes of every level


@pytest.fixture(scope="module")
def full():
    banner("fullsize: 1024^3 step")
    vol = synth.make_volume(synth.FULL, dev())
    pipe = P.PreviewPipeline(vol.shape, P.PreviewConfig(), device=dev())
    pipe.samples.zero_()
    pipe.step(vol, count=True)
    torch.cuda.synchronize()
    a = u16_np(vol)
    del vol
    torch.cuda.empty_cache()
    H, Ht = O.histogram(a), O.histogram(a, 0, 3)
    T = O.valley_threshold(H)
    return pipe, a, H, Ht, T, O.keep_bits(T, Ht)


def test_histograms(full):
    pipe, a, H, Ht, T, bits = full
    banner("fullsize: histograms")
    assert int(H.sum()) == a.size
    assert np.array_equal(u64_np(pipe.hist), H)
    assert np.array_equal(u64_np(pipe.hist_top), Ht)


def test_threshold_and_mask(full):
    pipe, a, H, Ht, T, bits = full
    banner(f"fullsize: threshold {T}")
    assert int(pipe.result[0].item()) == T
    assert np.array_equal(u32_np(pipe.keep), bits)
    # the threshold separates air from the outer shell of the generated scene
    assert 1000 + 3 * 40 < T < 8000 - 3 * 300


def test_levels_on_sampled_slabs(full):
    pipe, a, H, Ht, T, bits = full
    rng = np.random.default_rng(7)
    n_slabs = a.shape[0] // SLAB
    slabs = sorted(set(rng.choice(n_slabs, size=6, replace=False).tolist()) | {0, n_slabs - 1})
    for s in slabs:
        banner(f"fullsize: levels of slab {s}")
        ref = O.pyramid(a[SLAB * s:SLAB * (s + 1)], bits, 4)
        for k in range(1, 5):
            z0, z1 = (SLAB * s) >> k, (SLAB * (s + 1)) >> k
            got = u16_np(pipe.levels[k - 1][z0:z1].contiguous())
            assert np.array_equal(got, ref[k - 1]), (s, k)


def test_atlas_is_slicemap_of_level2(full):
    pipe, *_ = full
    banner("fullsize: atlas")
    L2 = u16_np(pipe.levels[1])
    tx, ty = pipe.tiles
    assert np.array_equal(u16_np(pipe.atlas), O.slicemap(L2, tx, ty, 16))


@pytest.fixture(scope="module")
def level1(full):
    pipe, a, H, Ht, T, bits = full
    banner("fullsize: oracle level 1, slab by slab")
    nz = a.shape[0]
    out = np.empty(O.level_dims(a.shape[2], a.shape[1], nz, 1)[::-1], dtype=np.uint16)
    for z in range(0, nz, SLAB):
        out[z // 2:(z + SLAB) // 2] = O.pyramid(a[z:z + SLAB], bits, 1)[0]
    return out


def test_level1_in_full(full, level1):
    pipe, *_ = full
    banner("fullsize: level 1 in full")
    assert np.array_equal(u16_np(pipe.levels[0]), level1)


@pytest.fixture(scope="module")
def oracle_frames(full, level1):
    pipe, *_ = full
    c = pipe.cfg
    banner(f"fullsize: FP64 oracle of all {len(pipe.cams)} x {c.width}x{c.height} frames")
    return R.render(level1, (1, 1, 1), pipe.tf.cpu().numpy().astype(np.float64), pipe.cams,
                    c.width, c.height, c.step, c.ert_eps, bounds=True)


def test_frames_in_full(full, oracle_frames):
    """Every pixel of the 36 turntable frames within 2e-4 of the FP64 oracle,
    which renders them from its own level 1."""
    pipe, *_ = full
    banner("fullsize: frames in full")
    ref, _, _ = oracle_frames
    err = float(np.abs(pipe.frames.cpu().numpy() - ref).max())
    assert err <= 2e-4, err
    assert ref[..., 3].max() > 0.5                        # the frames see the specimen


def test_headline_sample_count(full, oracle_frames):
    """The samples the 1024^3 step counts (the throughput's numerator) against
    the oracle's count of samples taken before early termination: within the
    per-ray bounds of an FP32 decision on the step count or the termination
    sample (L/step within 2^-10 of an integer, T within a factor 1 -/+ 2^-10
    of the threshold)."""
    pipe, *_ = full
    _, n_ref, lohi = oracle_frames
    n_gpu = int(pipe.samples[0].item())
    n_or, lo, hi = int(n_ref.sum()), int(lohi[:, 0].sum()), int(lohi[:, 1].sum())
    banner(f"fullsize: samples gpu {n_gpu} oracle {n_or} bounds [{lo}, {hi}]")
    assert lo <= n_gpu <= hi, (n_gpu, n_or, lo, hi)
    assert hi - lo <= 1e-3 * n_or                         # the bounds are tight
    assert int(pipe.samples[1].item()) <= n_gpu           # evaluated <= taken


def test_staged_march_at_full_size(full):
    """The depth-window march with LDS staging (on plain 4^3 bricks of the level, marked
    like the step's) renders the step's 36 frames bit for bit like the gather march the
    step uses, and takes as many samples."""
    from paper_2311_15038_amd import vr
    pipe, *_ = full
    c = pipe.cfg
    banner("fullsize: staged march")
    b4 = vr.vr_brick_volume(pipe.levels[c.render_level - 1], mark_above=pipe.mark_above)
    cnt = torch.zeros(2, dtype=torch.int64, device=dev())
    img = vr.vr_raycast(b4, pipe.tf, pipe.cams, c.width, c.height, c.step, ert_eps=c.ert_eps,
                        samples=cnt, staged=True)
    assert torch.equal(img, pipe.frames)
    assert int(cnt[0]) == int(pipe.samples[0])


@pytest.mark.parametrize("shift", [8, 0])
def test_otsu_and_its_full_histogram(full, shift):
    """Algorithms 1 and 2 on the full volume's histogram, on 256 (8-bit) and 65536 bins."""
    from paper_2311_15038_amd import vr
    pipe, a, H, Ht, T, bits = full
    banner(f"fullsize: otsu / its shift {shift}")
    Hc = H.reshape(-1, 1 << shift).sum(axis=1)
    res, _ = vr.vr_select_threshold(pipe.hist, None, vr.RULE_OTSU, shift)
    assert int(res[0].item()) == O.otsu_threshold(Hc) << shift
    res, _ = vr.vr_select_threshold(pipe.hist, None, vr.RULE_ITS, shift)
    Ti, it = O.its_threshold(Hc)
    assert int(res[0].item()) == Ti << shift and int(res[1].item()) == it
