"""Fitting a coarse preview grid and the transfer function to target renders
(projected Adam through the differentiable ray caster), with checkpoint and
resume.

The state is the density grid, the transfer-function table, the optimizer's
moments and the step count; `save` writes it with torch.save and `load` reads
it back with weights_only=True.  A resumed fit takes the same steps as one
that was never interrupted, up to the order of the density-gradient atomics.
"""
from __future__ import annotations

import copy

import torch

from . import autograd as VA


class PreviewFit:
    def __init__(self, density, tf, cams, width, height, step, target, spacing=(1.0, 1.0, 1.0), lr=1e-3,
                 fused=True):
        """density: f32 [nz][ny][nx] initial grid; tf: f32 [256][4] initial table;
        target: f32 [views][height][width][4] renders to fit (all on one device)."""
        self.density = density.detach().to(torch.float32).contiguous().clone().requires_grad_(True)
        self.tf = tf.detach().to(torch.float32).contiguous().clone().requires_grad_(True)
        self.cams, self.width, self.height, self.step_len = cams, width, height, step
        self.spacing = tuple(spacing)
        self.target = target
        self.opt = torch.optim.Adam([self.density, self.tf], lr=lr, fused=fused)
        self.steps = 0

    def step(self) -> torch.Tensor:
        """One iteration: forward, loss (mean squared error), adjoint, Adam, then the
        projection (densities in [0, 1], TF entries non-negative).  Returns the loss
        (a device tensor, no host synchronisation)."""
        self.opt.zero_grad(set_to_none=False)
        img = VA.render(self.density, self.tf, self.cams, self.width, self.height, self.step_len, self.spacing)
        loss = ((img - self.target) ** 2).mean()
        loss.backward()
        self.opt.step()
        with torch.no_grad():
            self.density.clamp_(0.0, 1.0)
            self.tf.clamp_(min=0.0)
        self.steps += 1
        return loss.detach()

    def state_dict(self) -> dict:
        """A snapshot: later steps do not change it (the optimizer's own state_dict
        holds references to its live moments, so it is copied)."""
        return {"density": self.density.detach().clone(), "tf": self.tf.detach().clone(),
                "adam": copy.deepcopy(self.opt.state_dict()), "steps": self.steps}

    def load_state_dict(self, state: dict) -> None:
        with torch.no_grad():
            self.density.copy_(state["density"])
            self.tf.copy_(state["tf"])
        self.opt.load_state_dict(state["adam"])
        self.steps = int(state["steps"])

    def save(self, path) -> None:
        torch.save(self.state_dict(), path)

    def load(self, path) -> None:
        self.load_state_dict(torch.load(path, map_location=self.density.device, weights_only=True))
