"""Batched persistent launch: every item equals its single-volume result.

Reduction outputs (threshold, level 1) bit-exact; frames bit-identical to the
single-volume ray caster on the same bricked level and within 2e-4 of the
oracle; repeated launches and HIP graph replays give the same results; other
launch shapes (the tuner's choices, down to the smallest tasks, which split
every histogram over many tasks) do not change them.  A batch of volumes at
the extremes of the uneven-batch sizes (64 to 512 voxels per axis) is checked
against the oracle too.
"""
import json

import numpy as np
import pytest
import torch

from oracle import reduce as O
from oracle import render as R
from paper_2311_15038_amd import batch as VB
from paper_2311_15038_amd import synth, vr

from gpu_util import banner, dev, u16_np

pytestmark = pytest.mark.gpu

SHAPES = [(29, 50, 37), (64, 48, 80), (40, 40, 40), (17, 33, 71), (96, 64, 72)]   # (nz, ny, nx)


@pytest.fixture(scope="module")
def volumes():
    out = []
    for k, (nz, ny, nx) in enumerate(SHAPES):
        out.append(synth.make_volume(synth.scaled_spec(nx, ny, nz, 4000 + k), dev()))
    return out


def _solo(v, cams, W, H, tf):
    Hh, Ht = vr.vr_histogram_with_top(v, 3)
    res, bits = vr.vr_select_threshold(Hh, Ht, vr.RULE_VALLEY, 32)
    (L1,) = vr.vr_threshold_downsample(v, bits, 1)
    bv = vr.vr_brick_volume(L1)
    fr = vr.vr_raycast(bv, tf, cams, W, H, 0.5)
    return res, L1, fr


def test_batch_matches_single_volume(volumes):
    banner("batch vs solo")
    W = H = 40
    b = VB.BatchPreview(volumes, n_views=3, width=W, height=H)
    b.launch()
    torch.cuda.synchronize()
    st, (taken, evald) = b.status()
    assert st == 0 and taken > 0 and 0 < evald <= taken
    for i, v in enumerate(volumes):
        res, L1, fr = _solo(v, b.cams[i][0], W, H, b.tf)
        assert b.result(i)[0].item() == res[0].item()
        assert torch.equal(b.level1(i), L1)
        assert torch.equal(b.frames[i], fr)
    b.close()


@pytest.mark.parametrize("hist_task_voxels,brick_edge", [(4 << 20, 4), (8192, 4), (4 << 20, 8)])
def test_batch_matches_oracle(volumes, hist_task_voxels, brick_edge):
    banner(f"batch vs oracle, {hist_task_voxels} voxels per histogram task, {brick_edge}^3 bricks")
    W = H = 24
    b = VB.BatchPreview(volumes[:3], n_views=2, width=W, height=H,
                        tuning=dict(hist_task_voxels=hist_task_voxels, brick_edge=brick_edge))
    b.launch()
    torch.cuda.synchronize()
    tf = synth.default_tf().astype(np.float64)
    for i, v in enumerate(volumes[:3]):
        a = u16_np(v)
        Hh, Ht = O.histogram(a), O.histogram(a, 0, 3)
        T = O.valley_threshold(Hh)
        L1 = O.pyramid(a, O.keep_bits(T, Ht), 1)[0]
        assert b.result(i)[0].item() == T
        assert (u16_np(b.level1(i)) == L1).all()
        ref, _ = R.render(L1, (1, 1, 1), tf, b.cams[i][0], W, H, 0.5)
        assert np.abs(b.frames[i].cpu().numpy() - ref).max() <= 2e-4
    b.close()


def test_batch_relaunch_and_graph_replay(volumes):
    banner("batch relaunch + graph replay")
    b = VB.BatchPreview(volumes, n_views=2, width=32, height=32)
    b.launch()
    torch.cuda.synchronize()
    first = [f.clone() for f in b.frames]
    lv = [b.level1(i).clone() for i in range(len(volumes))]
    for f in b.frames:
        f.zero_()
    b.launch()                                    # the queue and counters reset themselves
    torch.cuda.synchronize()
    assert all(torch.equal(a, f) for a, f in zip(first, b.frames))
    b.capture()
    for rep in range(3):
        for f in b.frames:
            f.fill_(float(rep + 1))               # eager work between replays
        torch.cuda.synchronize()
        b.launch()
        torch.cuda.synchronize()
        assert all(torch.equal(a, f) for a, f in zip(first, b.frames)), rep
        assert all(torch.equal(a, b.level1(i)) for i, a in enumerate(lv))
    assert b.status()[0] == 0
    b.close()


def test_launch_shape_does_not_change_results(volumes):
    banner("batch tunings agree")
    ref = None
    for t in [dict(wave_w=8, wave_h=8, waves_x=4), dict(wave_w=16, wave_h=4, waves_x=2, hist_task_voxels=1 << 20,
                                                       down_tiles_per_task=3, slabs_per_task=5),
              dict(wave_w=4, wave_h=16, waves_x=8, down_tiles_per_task=64, slabs_per_task=200),
              dict(hist_task_voxels=8192, down_tiles_per_task=1, slabs_per_task=1),
              dict(brick_edge=8), dict(brick_edge=8, slabs_per_task=1, wave_w=16, wave_h=4, waves_x=2)]:
        b = VB.BatchPreview(volumes, n_views=2, width=35, height=29, tuning=t)
        b.launch()
        torch.cuda.synchronize()
        out = [f.clone() for f in b.frames]
        assert b.status()[0] == 0
        b.close()
        if ref is None:
            ref = out
        else:
            assert all(torch.equal(a, c) for a, c in zip(ref, out))


def test_tuner_runs(volumes, tmp_path, monkeypatch):
    banner("tuner")
    monkeypatch.setenv("VR_AUTOTUNE_CACHE", str(tmp_path / "cache.json"))
    best, timings = VB.tune(volumes[:2], n_views=2, width=32, height=32)
    # every render tile is timed; brick sizes and task sizes too (a repeat of a timed
    # configuration counts once)
    assert len(VB.RENDER_TILES) <= len(timings) <= len(VB.RENDER_TILES) + len(VB.BRICK_EDGES) + len(VB.TASK_SIZES)
    assert best["brick_edge"] in VB.BRICK_EDGES
    assert json.loads(min(timings, key=timings.get)) == best
    again, t2 = VB.tune(volumes[:2], n_views=2, width=32, height=32)
    assert again == best and t2 == {}              # served from the cache


def test_batch_rejects_bad_config(volumes):
    with pytest.raises(vr.VrError):
        VB.BatchPreview(volumes[:1], n_views=2, width=8, height=8, tuning=dict(wave_w=8, wave_h=4))
    with pytest.raises(vr.VrError):
        VB.BatchPreview(volumes[:1], n_views=49, width=8, height=8)


# (nz, ny, nx) at the extremes of 64..512 per axis, plus a ragged one
CONFIG3_SHAPES = [(384, 64, 512), (64, 512, 512), (512, 512, 64), (64, 64, 64), (301, 77, 449)]


def test_batch_extreme_shapes_match_oracle():
    """Volumes at the extremes of the uneven-batch sizes: with the default task
    sizes the larger ones take several histogram tasks each (4 Mi voxels per
    task), whose counts are summed into one histogram.  Thresholds and level 1
    bit-exact against the oracle, frames bit-identical to the single-volume path
    and within 2e-4 of the oracle."""
    vols = [synth.make_volume(synth.scaled_spec(nx, ny, nz, 4100 + k), dev())
            for k, (nz, ny, nx) in enumerate(CONFIG3_SHAPES)]
    W = H = 48
    banner(f"batch of extreme shapes {CONFIG3_SHAPES}")
    b = VB.BatchPreview(vols, n_views=3, width=W, height=H)
    b.launch()
    torch.cuda.synchronize()
    assert b.status()[0] == 0
    assert b.n_tasks() > 2 * len(vols)
    tf = synth.default_tf().astype(np.float64)
    for i, v in enumerate(vols):
        banner(f"extreme shape {tuple(v.shape)}: oracle")
        a = u16_np(v)
        Hh, Ht = O.histogram(a), O.histogram(a, 0, 3)
        T = O.valley_threshold(Hh)
        L1 = O.pyramid(a, O.keep_bits(T, Ht), 1)[0]
        assert b.result(i)[0].item() == T, (i, b.result(i)[0].item(), T)
        assert np.array_equal(u16_np(b.level1(i)), L1), i
        res, L1g, fr = _solo(v, b.cams[i][0], W, H, b.tf)
        assert torch.equal(b.frames[i], fr), i
        ref, _ = R.render(L1, (1, 1, 1), tf, b.cams[i][0], W, H, 0.5)
        err = float(np.abs(b.frames[i].cpu().numpy() - ref).max())
        assert err <= 2e-4, (i, err)
    b.close()
