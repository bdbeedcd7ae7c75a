"""The single-volume brick-size tuner: it times both brick sizes on the
pipeline's own level, caches its choice, and either choice renders the same
frames (bit-identical) as the other."""
import pytest
import torch

from paper_2311_15038_amd import pipeline as P
from paper_2311_15038_amd import synth

from gpu_util import banner, dev

pytestmark = pytest.mark.gpu


def test_brick_edge_tuner(tmp_path, monkeypatch):
    banner("single-volume brick-size tuner")
    monkeypatch.setenv("VR_AUTOTUNE_CACHE", str(tmp_path / "cache.json"))
    vol = synth.make_volume(synth.scaled_spec(150, 128, 96, 4200), dev())
    cfg = P.PreviewConfig(n_levels=2, atlas_level=0, n_views=6, width=96, height=80)
    pipe = P.PreviewPipeline(vol.shape, cfg, device=dev())
    pipe.step(vol)
    edge, times = P.tune_brick_edge(pipe)
    assert edge in (4, 8) and set(times) == {4, 8} and times[edge] == min(times.values())
    again, t2 = P.tune_brick_edge(pipe)
    assert again == edge and t2 == {}                  # served from the cache
    frames = {}
    for e in (4, 8):
        p = P.PreviewPipeline(vol.shape, P.PreviewConfig(n_levels=2, atlas_level=0, n_views=6, width=96,
                                                         height=80, brick_edge=e), device=dev())
        p.step(vol, count=True)
        torch.cuda.synchronize()
        frames[e] = (p.frames.clone(), p.samples.clone(), p.view_hist.clone())
    assert torch.equal(frames[4][0], frames[8][0])
    assert int(frames[4][1][0]) == int(frames[8][1][0])
    assert torch.equal(frames[4][2], frames[8][2])
