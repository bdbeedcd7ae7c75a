"""The fit's checkpoint logic on the host (no rendering): state_dict is a
snapshot that later optimizer steps leave alone, and save/load restores grid,
transfer function, Adam moments and step count bit for bit through a file
read back with weights_only=True."""
import os

import torch

from paper_2311_15038_amd import fit as VF


def _fit(seed):
    g = torch.Generator().manual_seed(seed)
    dens = torch.rand((6, 5, 4), generator=g)
    tf = torch.rand((256, 4), generator=g)
    f = VF.PreviewFit(dens, tf, cams=None, width=4, height=4, step=1.0, target=None, lr=1e-2, fused=False)
    return f, g


def _adam_step(f, g):
    """One optimizer step on random gradients (what `step` does after the adjoint)."""
    f.density.grad = torch.randn(f.density.shape, generator=g)
    f.tf.grad = torch.randn(f.tf.shape, generator=g)
    f.opt.step()
    f.steps += 1


def test_state_dict_is_a_snapshot():
    f, g = _fit(1)
    for _ in range(3):
        _adam_step(f, g)
    snap = f.state_dict()
    m = [s["exp_avg"].clone() for s in snap["adam"]["state"].values()]
    d = snap["density"].clone()
    _adam_step(f, g)
    assert snap["steps"] == 3 and f.steps == 4
    assert torch.equal(snap["density"], d)
    for a, s in zip(m, snap["adam"]["state"].values()):
        assert torch.equal(a, s["exp_avg"])
    live = list(f.opt.state_dict()["state"].values())
    assert not torch.equal(live[0]["exp_avg"], m[0])


def test_save_and_load_round_trip(tmp_path):
    a, g = _fit(2)
    for _ in range(5):
        _adam_step(a, g)
    path = os.path.join(tmp_path, "fit.pt")
    a.save(path)
    b, _ = _fit(3)
    b.load(path)
    assert b.steps == 5
    assert torch.equal(a.density, b.density) and torch.equal(a.tf, b.tf)
    sa, sb = a.opt.state_dict(), b.opt.state_dict()
    assert sa["param_groups"] == sb["param_groups"]
    for x, y in zip(sa["state"].values(), sb["state"].values()):
        for key in ("exp_avg", "exp_avg_sq", "step"):
            assert torch.equal(x[key], y[key]), key
    # the same gradients take both to the same place
    ga, gb = torch.Generator().manual_seed(9), torch.Generator().manual_seed(9)
    _adam_step(a, ga)
    _adam_step(b, gb)
    assert torch.equal(a.density, b.density) and torch.equal(a.tf, b.tf)
