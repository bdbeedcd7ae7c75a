"""Checkpoint and resume of the preview fit: a fit saved after 6 steps and
loaded into a fresh object takes the same next steps as the uninterrupted
one.  The saved state comes back bit for bit; the steps after it agree up to
the order of the density-gradient atomics."""
import os

import numpy as np
import pytest
import torch

from paper_2311_15038_amd import fit as VF
from paper_2311_15038_amd import synth, vr

from gpu_util import banner, dev

pytestmark = pytest.mark.gpu


def _problem():
    n = 32
    rng = np.random.default_rng(9)
    idx = np.indices((n, n, n)).astype(np.float64)
    truth = np.clip(0.4 * np.exp(-((idx - n / 2) ** 2).sum(axis=0) / (2 * (n / 5) ** 2)), 0, 1)
    tf = torch.from_numpy(synth.default_tf(sigma_scale=3.0)).to(dev())
    cams = synth.turntable_cameras(n, n, n, n_views=6)
    target = vr.vr_raycast(torch.tensor(truth, dtype=torch.float32, device=dev()), tf, cams, 40, 40, 0.5)
    init = torch.tensor(0.05 + 0.05 * rng.random((n // 2,) * 3), dtype=torch.float32, device=dev())
    return init, tf, cams, target


def _fit(init, tf, cams, target):
    return VF.PreviewFit(init, tf, cams, 40, 40, 1.0, target, spacing=(2.0, 2.0, 2.0), lr=1e-2)


def test_resume_from_checkpoint(tmp_path):
    banner("fit: checkpoint after 6 steps, resume, 6 more")
    init, tf, cams, target = _problem()
    a = _fit(init, tf, cams, target)
    la = [float(a.step().item()) for _ in range(6)]
    path = os.path.join(tmp_path, "fit.pt")
    a.save(path)
    saved = a.state_dict()
    la += [float(a.step().item()) for _ in range(6)]

    b = _fit(init, tf, cams, target)
    b.load(path)
    assert b.steps == 6
    assert torch.equal(b.density, saved["density"]) and torch.equal(b.tf, saved["tf"])
    for ga, gb in zip(saved["adam"]["state"].values(), b.opt.state_dict()["state"].values()):
        for key in ("exp_avg", "exp_avg_sq", "step"):
            assert torch.equal(ga[key].to(gb[key].device), gb[key]), key
    lb = [float(b.step().item()) for _ in range(6)]
    assert b.steps == 12
    assert np.allclose(lb, la[6:], rtol=1e-3, atol=0.0), (lb, la[6:])
    assert la[-1] < la[0]
    assert (b.density - a.density).abs().max().item() < 1e-3
