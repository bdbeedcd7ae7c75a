"""Differentiable FP64 reference of the emission-absorption ray caster.

TEST INFRASTRUCTURE ONLY.  A second, independent implementation of the
oracle's rendering model (the one in render.c), written with torch CPU
tensor ops in float64 and vectorised over rays, so that torch autograd gives
exact derivatives of the discrete sum with respect to the density grid and
the transfer-function table.  It marches every ray to its exit (no early
termination).  render() is vectorised over rays and steps one at a time, for
small grids (the autograd graph keeps every step's gathers of the grid);
march_rays() takes all samples of a few rays at once, for large grids.
"""
from __future__ import annotations

import math

import numpy as np
import torch


def rays(cams, W, H):
    """Origins and unit directions [V*H*W][3] (float64 numpy), pixel centres, row 0 on top."""
    cams = np.asarray(cams, dtype=np.float64).reshape(-1, 11)
    jj, ii = np.meshgrid(np.arange(H, dtype=np.float64), np.arange(W, dtype=np.float64),
                         indexing="ij")
    nx_ = (2.0 * (ii + 0.5) / W - 1.0) * (W / H)
    ny_ = 1.0 - 2.0 * (jj + 0.5) / H
    O, D = [], []
    for c in cams:
        eye, tgt, up = c[0:3], c[3:6], c[6:9]
        f = tgt - eye
        f = f / np.linalg.norm(f)
        r = np.cross(f, up)
        r = r / np.linalg.norm(r)
        u = np.cross(r, f)
        off = nx_[..., None] * r + ny_[..., None] * u
        if c[9] > 0:
            d = f + math.tan(math.radians(c[9]) / 2.0) * off
            d = d / np.linalg.norm(d, axis=-1, keepdims=True)
            o = np.broadcast_to(eye, d.shape)
        else:
            o = eye + c[10] * off
            d = np.broadcast_to(f, o.shape)
        O.append(o.reshape(-1, 3))
        D.append(d.reshape(-1, 3))
    return np.concatenate(O), np.concatenate(D)


def _clip(o, d, ext, step):
    """Entry distance t_in, clipped length L and step count n per ray (0 for a miss)."""
    # slab test per axis for the entry; the length from the entry point to the
    # first exit face (t_out - t_in without the cancellation of two long distances)
    with np.errstate(divide="ignore", invalid="ignore"):
        ta = (0.0 - o) / d
        tb = (ext - o) / d
    outside = ((d == 0.0) & ((o < 0.0) | (o > ext))).any(axis=1)
    lo = np.where(d == 0.0, -np.inf, np.minimum(ta, tb))
    t_in = np.where(outside, 0.0, np.maximum(lo.max(axis=1), 0.0))
    p_in = o + t_in[:, None] * d
    with np.errstate(divide="ignore", invalid="ignore"):
        la = np.where(d == 0.0, np.inf, (np.where(d > 0.0, ext, 0.0) - p_in) / d)
    Lr = np.where(outside, -np.inf, la.min(axis=1))
    hit = Lr > 0.0
    Lr = np.where(hit, Lr, 0.0)
    t_in = np.where(hit, t_in, 0.0)
    n = np.where(hit, np.maximum(1, np.ceil(Lr / step)), 0).astype(np.int64)
    return t_in, Lr, n


def render(density: torch.Tensor, tf: torch.Tensor, cams, W, H, step, spacing=(1.0, 1.0, 1.0),
           bg=(0.0, 0.0, 0.0, 0.0)) -> torch.Tensor:
    """rgba [V][H][W][4] as a differentiable function of density [nz][ny][nx] and tf [256][4]."""
    assert density.dtype == torch.float64 and tf.dtype == torch.float64
    nz, ny, nx = density.shape
    sp = np.asarray(spacing, dtype=np.float64)
    ext = np.array([nx, ny, nz], dtype=np.float64) * sp
    o, d = rays(cams, W, H)
    R = o.shape[0]
    t_in, Lr, n = _clip(o, d, ext, step)
    nmax = int(n.max()) if R else 0

    flat = density.reshape(-1)
    dims = np.array([nx, ny, nz])
    T = torch.ones(R, dtype=torch.float64)
    Cc = torch.zeros(R, 3, dtype=torch.float64)
    o_t, d_t = torch.from_numpy(o.copy()), torch.from_numpy(d.copy())
    t_in_t = torch.from_numpy(t_in)
    n_t = torch.from_numpy(n)
    L_t = torch.from_numpy(Lr)
    sp_t = torch.from_numpy(sp)
    for k in range(nmax):
        active = n_t > k
        last = n_t - 1 == k
        seg = torch.where(last, L_t - (n_t - 1).double() * step, torch.full_like(L_t, step))
        seg = torch.where(active, seg, torch.zeros_like(seg))
        t = torch.where(active, t_in_t + k * step + 0.5 * seg, torch.zeros_like(seg))
        p = o_t + t[:, None] * d_t
        u = p / sp_t - 0.5
        i0 = torch.floor(u)
        w = u - i0
        i0 = i0.long()
        s = torch.zeros(R, dtype=torch.float64)
        for dz in (0, 1):
            for dy in (0, 1):
                for dx in (0, 1):
                    xi = (i0[:, 0] + dx).clamp(0, int(dims[0]) - 1)
                    yi = (i0[:, 1] + dy).clamp(0, int(dims[1]) - 1)
                    zi = (i0[:, 2] + dz).clamp(0, int(dims[2]) - 1)
                    wt = ((w[:, 0] if dx else 1 - w[:, 0]) * (w[:, 1] if dy else 1 - w[:, 1])
                          * (w[:, 2] if dz else 1 - w[:, 2]))
                    s = s + wt * flat[(zi * ny + yi) * nx + xi]
        x = s.clamp(0.0, 1.0) * 255.0
        kk = torch.floor(x).long().clamp(max=254)
        ww = (x - kk.double())[:, None]
        q = (1 - ww) * tf[kk] + ww * tf[kk + 1]
        e = torch.exp(-q[:, 3] * seg)
        alpha = 1.0 - e
        Cc = Cc + (T * alpha)[:, None] * q[:, :3]
        T = T * e
    bg_t = torch.tensor(bg, dtype=torch.float64)
    rgb = Cc + T[:, None] * bg_t[:3]
    a = 1.0 - T * (1.0 - bg_t[3])
    out = torch.cat([rgb, a[:, None]], dim=1)
    V = len(np.asarray(cams).reshape(-1, 11))
    return out.reshape(V, H, W, 4)


def pixel_rays(cams, W, H, pix):
    """Origins and unit directions of the pixels pix[k] = (view, row j, column i)."""
    pix = np.asarray(pix, dtype=np.int64).reshape(-1, 3)
    o, d = rays(cams, W, H)
    idx = (pix[:, 0] * H + pix[:, 1]) * W + pix[:, 2]
    return o[idx], d[idx]


def march_rays(density: torch.Tensor, tf: torch.Tensor, o, d, step, spacing=(1.0, 1.0, 1.0),
               bg=(0.0, 0.0, 0.0, 0.0)) -> torch.Tensor:
    """rgba [R][4] of the rays (o, d), float64 numpy [R][3] with unit d: the model of
    render() written as one expression over every (ray, sample) pair, for a few
    hundred rays through a large grid.  Each of the eight taps is one gather over
    all samples (autograd then keeps eight gathers of the grid, not eight per step),
    the transmittance before sample i is the running product of the factors
    exp(-sigma_k len_k) of the samples before it, and the colour is the sum over
    samples of T_i (1 - exp(-sigma_i len_i)) rgb_i.  Samples past a ray's last have
    length 0 and add nothing."""
    assert density.dtype == torch.float64 and tf.dtype == torch.float64
    nz, ny, nx = density.shape
    sp = np.asarray(spacing, dtype=np.float64)
    ext = np.array([nx, ny, nz], dtype=np.float64) * sp
    o = np.ascontiguousarray(o, dtype=np.float64).reshape(-1, 3)
    d = np.ascontiguousarray(d, dtype=np.float64).reshape(-1, 3)
    R = o.shape[0]
    t_in, Lr, n = _clip(o, d, ext, step)
    nmax = max(int(n.max()) if R else 0, 1)
    k = np.arange(nmax, dtype=np.float64)[None, :]
    nn = n[:, None]
    seg = np.where(k < nn - 1, step, np.where(k == nn - 1, Lr[:, None] - (nn - 1) * step, 0.0))
    t = t_in[:, None] + k * step + 0.5 * seg
    p = o[:, None, :] + t[..., None] * d[:, None, :]            # [R][nmax][3]
    u = torch.from_numpy(p / sp - 0.5)
    i0 = torch.floor(u)
    w = u - i0
    i0 = i0.long()
    flat = density.reshape(-1)
    s = torch.zeros(R, nmax, dtype=torch.float64)
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                xi = (i0[..., 0] + dx).clamp(0, nx - 1)
                yi = (i0[..., 1] + dy).clamp(0, ny - 1)
                zi = (i0[..., 2] + dz).clamp(0, nz - 1)
                wt = ((w[..., 0] if dx else 1 - w[..., 0]) * (w[..., 1] if dy else 1 - w[..., 1])
                      * (w[..., 2] if dz else 1 - w[..., 2]))
                s = s + wt * flat[(zi * ny + yi) * nx + xi]
    x = s.clamp(0.0, 1.0) * 255.0
    kk = torch.floor(x).long().clamp(max=254)
    ww = (x - kk.double())[..., None]
    q = (1 - ww) * tf[kk] + ww * tf[kk + 1]                     # [R][nmax][4]
    e = torch.exp(-q[..., 3] * torch.from_numpy(seg))
    T_before = torch.cumprod(torch.cat([torch.ones(R, 1, dtype=torch.float64), e[:, :-1]], dim=1), dim=1)
    Cc = ((T_before * (1.0 - e))[..., None] * q[..., :3]).sum(dim=1)
    T = T_before[:, -1] * e[:, -1]
    bg_t = torch.tensor(bg, dtype=torch.float64)
    rgb = Cc + T[:, None] * bg_t[:3]
    a = 1.0 - T * (1.0 - bg_t[3])
    return torch.cat([rgb, a[:, None]], dim=1)
