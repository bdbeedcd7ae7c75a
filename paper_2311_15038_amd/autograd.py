"""torch.autograd.Function around the HIP ray caster and its adjoint.

The forward saves only its RGBA output; the backward re-marches every ray
(per-ray recomputation, nothing stored per sample) and scatters gradients to
the density grid and the transfer-function table.
"""
from __future__ import annotations

import numpy as np
import torch

from . import vr


class VolumeRender(torch.autograd.Function):
    @staticmethod
    def forward(ctx, density, tf, cams, width, height, step, spacing=(1.0, 1.0, 1.0),
                ert_eps=2.0 ** -14, bg=(0.0, 0.0, 0.0, 0.0)):
        if density.dtype != torch.float32:
            raise TypeError("VolumeRender differentiates an f32 density grid")
        density = density.contiguous()
        tf = tf.contiguous()
        out = vr.vr_raycast(density, tf, cams, width, height, step, spacing, ert_eps, bg)
        ctx.save_for_backward(density, tf, out)
        ctx.args = (np.asarray(cams, dtype=np.float64).copy(), width, height, step, spacing,
                    ert_eps, bg)
        return out

    @staticmethod
    def backward(ctx, grad_out):
        density, tf, out = ctx.saved_tensors
        cams, width, height, step, spacing, ert_eps, bg = ctx.args
        g_density = torch.zeros_like(density)
        g_tf = torch.zeros_like(tf)
        vr.vr_raycast_backward(density, tf, cams, width, height, step, out, grad_out.contiguous(),
                               g_density, g_tf, spacing, ert_eps, bg)
        return g_density, g_tf, None, None, None, None, None, None, None


def render(density, tf, cams, width, height, step, spacing=(1.0, 1.0, 1.0), ert_eps=2.0 ** -14,
           bg=(0.0, 0.0, 0.0, 0.0)):
    return VolumeRender.apply(density, tf, cams, width, height, step, spacing, ert_eps, bg)
