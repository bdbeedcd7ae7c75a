"""The single-volume preview step captured in a HIP graph (through torch's
CUDAGraph, which drives hipGraph capture on ROCm): every call is asynchronous
on the caller's stream and allocates nothing when its outputs are given, so
the whole step replays without the host.  Each replay is checked against the
eager step, with eager work on another volume and synchronisations between
the replays."""
import numpy as np
import pytest
import torch

from paper_2311_15038_amd import pipeline as P
from paper_2311_15038_amd import synth

from gpu_util import banner, dev

pytestmark = pytest.mark.gpu

OUTPUTS = ("hist", "hist_top", "result", "keep", "atlas", "frames", "view_hist", "view_entropy", "best_view")


def _snapshot(pipe):
    out = {k: getattr(pipe, k).clone() for k in OUTPUTS}
    out["levels"] = [lv.clone() for lv in pipe.levels]
    return out


def _equal(a, b):
    for k in OUTPUTS:
        assert torch.equal(a[k], b[k]), k
    for x, y in zip(a["levels"], b["levels"]):
        assert torch.equal(x, y)


def test_small_step_replays_from_a_graph():
    banner("graph: 128^3 preview step captured and replayed")
    vol = synth.make_volume(synth.SMALL, dev())
    other = synth.make_volume(synth.VolumeSpec(128, 128, 128, seed=77), dev())
    cfg = P.PreviewConfig(n_levels=2, atlas_level=1, render_level=1, n_views=3, width=128, height=128)
    pipe = P.PreviewPipeline(vol.shape, cfg, device=dev())
    side = P.PreviewPipeline(other.shape, cfg, device=dev())
    pipe.step(vol)
    torch.cuda.synchronize()
    ref = _snapshot(pipe)
    # warm up on a side stream, as capture requires, then capture one step
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        pipe.step(vol)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        pipe.step(vol)
    torch.cuda.synchronize()
    for r in range(4):
        # eager work of the same library between replays, and the outputs overwritten
        side.step(other)
        for k in ("frames", "atlas"):
            getattr(pipe, k).zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        _equal(_snapshot(pipe), ref)
        banner(f"graph: replay {r} matches the eager step")
    assert int(pipe.result[0].item()) == int(ref["result"][0].item())
    assert not np.array_equal(side.frames.cpu().numpy(), pipe.frames.cpu().numpy())
