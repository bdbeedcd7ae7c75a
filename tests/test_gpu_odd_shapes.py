"""An odd, anisotropic volume (x 511, y 257, z 129: no side a multiple of 2,
4, 16 or 32) through the whole preview step, against the oracle: histograms,
threshold, keep mask, eight pyramid levels (the last four summed from the
exact level-4 sums after the pass) and the atlas bit-exact, frames
within 2e-4 of the FP64 ray caster.  The step then runs again on the same
input and every output must come out bit for bit the same (the integer
outputs are deterministic, so a race in an LDS pass would show here)."""
import numpy as np
import pytest
import torch

from oracle import reduce as O
from oracle import render as R
from paper_2311_15038_amd import pipeline as P
from paper_2311_15038_amd import synth

from gpu_util import banner, dev, u16_np, u32_np, u64_np

pytestmark = pytest.mark.gpu

SHAPE = (129, 257, 511)


@pytest.fixture(scope="module")
def odd():
    nz, ny, nx = SHAPE
    banner(f"odd shape {SHAPE}: preview step")
    vol = synth.make_volume(synth.VolumeSpec(nx, ny, nz, seed=4242), dev())
    cfg = P.PreviewConfig(n_levels=8, atlas_level=2, render_level=1, n_views=2, width=72, height=40)
    pipe = P.PreviewPipeline(vol.shape, cfg, device=dev())
    pipe.step(vol)
    torch.cuda.synchronize()
    return pipe, vol, u16_np(vol)


def test_reduction_bit_exact(odd):
    pipe, _, a = odd
    H, Ht = O.histogram(a), O.histogram(a, 0, 3)
    assert np.array_equal(u64_np(pipe.hist), H) and np.array_equal(u64_np(pipe.hist_top), Ht)
    T = O.valley_threshold(H)
    bits = O.keep_bits(T, Ht)
    assert int(pipe.result[0].item()) == T and np.array_equal(u32_np(pipe.keep), bits)
    ref = O.pyramid(a, bits, 8)
    for k in range(8):
        assert np.array_equal(u16_np(pipe.levels[k]), ref[k]), k + 1
    tx, ty = pipe.tiles
    assert np.array_equal(u16_np(pipe.atlas), O.slicemap(ref[1], tx, ty, 16))


def test_frames_within_tolerance(odd):
    pipe, _, _ = odd
    level1 = u16_np(pipe.levels[0])
    ref, _ = R.render(level1, (1, 1, 1), pipe.tf.cpu().numpy().astype(np.float64), pipe.cams, 72, 40, 0.5)
    got = pipe.frames.cpu().numpy().astype(np.float64)
    assert np.abs(got - ref).max() <= 2e-4


def test_second_run_is_bit_identical(odd):
    pipe, vol, _ = odd
    first = {k: getattr(pipe, k).clone() for k in ("hist", "hist_top", "result", "keep", "atlas", "frames")}
    levels = [lv.clone() for lv in pipe.levels]
    pipe.step(vol)
    torch.cuda.synchronize()
    for k, v in first.items():
        assert torch.equal(getattr(pipe, k), v), k
    for a, b in zip(levels, pipe.levels):
        assert torch.equal(a, b)


def test_tf_marked_bricks_change_nothing(odd):
    """The step marks bricks above the level its TF leaves at zero extinction; the
    same step with bricks marked by every non-zero voxel gives the same frames,
    grey-value counts and taken samples bit for bit, and evaluates no fewer."""
    pipe, vol, _ = odd
    assert pipe.mark_above > 0
    cfg = P.PreviewConfig(n_levels=8, atlas_level=2, render_level=1, n_views=2, width=72, height=40,
                          mark_by_tf=False)
    plain = P.PreviewPipeline(vol.shape, cfg, device=dev())
    assert plain.mark_above == 0
    pipe.samples.zero_()
    plain.samples.zero_()
    pipe.step(vol, count=True)
    plain.step(vol, count=True)
    torch.cuda.synchronize()
    assert torch.equal(pipe.frames, plain.frames) and torch.equal(pipe.view_hist, plain.view_hist)
    assert pipe.samples[0].item() == plain.samples[0].item()
    assert pipe.samples[1].item() <= plain.samples[1].item()
