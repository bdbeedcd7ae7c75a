"""torch.autograd.Function around the HIP ray caster and its adjoint.

The forward saves only its RGBA output; the backward re-marches every ray
(per-ray recomputation, nothing stored per sample) and scatters gradients to
the density grid and the transfer-function table.

The forward renders from a 4^3-brick copy of the grid with empty-space
skipping: a skipped sample has zero extinction, so the frames (and the
sample where each ray terminates early) are bit-identical to marching the
linear grid.  The adjoint replays the same bricked copy, scatters the
density gradient in the brick layout (a cell's taps then share cache lines)
and brings it back to the grid's layout.  It passes over the same empty
bricks when the first TF segment has zero extinction, adding in closed form
the one gradient their samples carry (to that knot's extinction); otherwise
it marches every sample.
"""
from __future__ import annotations

import numpy as np
import torch

from . import vr


def render_forward(density, tf, cams, width, height, step, spacing=(1.0, 1.0, 1.0), ert_eps=2.0 ** -14,
                   bg=(0.0, 0.0, 0.0, 0.0), skip_empty=True, samples=None, with_occupancy=False,
                   with_source=False):
    """The frames of an f32 grid as the differentiable render's forward makes them
    (with with_occupancy, also the brick occupancy grid, or None; with with_source,
    also the grid it rendered: the bricked copy, or the grid itself)."""
    src = vr.vr_brick_volume(density) if skip_empty else density
    out = vr.vr_raycast(src, tf, cams, width, height, step, spacing, ert_eps, bg, samples=samples)
    extra = []
    if with_occupancy:
        extra.append(src.occupancy if skip_empty else None)
    if with_source:
        extra.append(src)
    return (out, *extra) if extra else out


class VolumeRender(torch.autograd.Function):
    @staticmethod
    def forward(ctx, density, tf, cams, width, height, step, spacing=(1.0, 1.0, 1.0),
                ert_eps=2.0 ** -14, bg=(0.0, 0.0, 0.0, 0.0), skip_empty=True):
        if density.dtype != torch.float32:
            raise TypeError("VolumeRender differentiates an f32 density grid")
        density = density.contiguous()
        tf = tf.contiguous()
        out, src = render_forward(density, tf, cams, width, height, step, spacing, ert_eps, bg, skip_empty,
                                  with_source=True)
        ctx.save_for_backward(density, tf, out)
        ctx.src = src
        ctx.args = (np.asarray(cams, dtype=np.float64).copy(), width, height, step, spacing,
                    ert_eps, bg)
        return out

    @staticmethod
    def backward(ctx, grad_out):
        density, tf, out = ctx.saved_tensors
        cams, width, height, step, spacing, ert_eps, bg = ctx.args
        src = ctx.src
        g_tf = torch.zeros_like(tf)
        if isinstance(src, vr.BrickedVolume):
            # the adjoint replays the bricked copy and scatters in its layout
            g_b = torch.zeros_like(src.data)
            vr.vr_raycast_backward(src, tf, cams, width, height, step, out, grad_out.contiguous(),
                                   g_b, g_tf, spacing, ert_eps, bg, occupancy=src.occupancy)
            g_density = vr.vr_unbrick_volume(vr.BrickedVolume(g_b, src.shape, None, src.layout))
        else:
            g_density = torch.zeros_like(density)
            vr.vr_raycast_backward(density, tf, cams, width, height, step, out, grad_out.contiguous(),
                                   g_density, g_tf, spacing, ert_eps, bg)
        ctx.src = None
        return g_density, g_tf, None, None, None, None, None, None, None, None


def render(density, tf, cams, width, height, step, spacing=(1.0, 1.0, 1.0), ert_eps=2.0 ** -14,
           bg=(0.0, 0.0, 0.0, 0.0), skip_empty=True):
    return VolumeRender.apply(density, tf, cams, width, height, step, spacing, ert_eps, bg, skip_empty)
