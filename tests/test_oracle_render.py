"""Pins for the FP64 ray-casting oracle (render.c) and its torch twin.

Closed forms (background, Beer-Lambert, a linear ramp the midpoint rule
integrates exactly), brute force on tiny scenes (tent-kernel density and a
hand-written march), symmetries, step refinement, and agreement of the two
independent FP64 implementations.
"""
import math

import numpy as np
import pytest
import torch

from oracle import render as R
from oracle import render_torch as RT
from paper_2311_15038_amd import synth


def _const_tf(rgb, sigma):
    tf = np.zeros((256, 4))
    tf[:, :3] = rgb
    tf[:, 3] = sigma
    return tf


def _linear_tf(rgb, c):
    tf = np.zeros((256, 4))
    tf[:, :3] = rgb
    tf[:, 3] = c * np.arange(256) / 255.0          # sigma(s) = c * s exactly
    return tf


BG = (0.25, 0.5, 0.125, 0.75)                    # exactly representable


def test_empty_volume_is_background():
    vol = np.zeros((9, 7, 5), dtype=np.uint16)
    cams = np.concatenate([synth.turntable_cameras(5, 7, 9, n_views=3),
                           synth.front_ortho_camera(5, 7, 9)])
    img, cnt = R.render(vol, (1, 1, 1), synth.default_tf(), cams, 16, 12, 0.5, bg=BG)
    assert (img == np.array(BG)).all()


def test_miss_is_background():
    vol = np.full((4, 4, 4), 30000, dtype=np.uint16)
    cam = synth.front_ortho_camera(4, 4, 4)
    cam[0, 0:3] += (100.0, 0.0, 0.0)                # looking past the box
    cam[0, 3:6] += (100.0, 0.0, 0.0)
    img, cnt = R.render(vol, (1, 1, 1), _const_tf(0.9, 1.0), cam, 8, 8, 0.5, bg=BG)
    assert (img == np.array(BG)).all() and cnt[0] == 0


@pytest.mark.parametrize("spacing", [(1, 1, 1), (1.0, 1.5, 0.5)])
def test_constant_slab_beer_lambert(spacing):
    nx, ny, nz = 6, 10, 8
    vol = np.full((nz, ny, nx), 20000, dtype=np.uint16)
    rgb, sig = np.array([0.7, 0.2, 0.4]), 0.13
    cam = synth.front_ortho_camera(nx, ny, nz, spacing)
    img, _ = R.render(vol, spacing, _const_tf(rgb, sig), cam, 9, 7, 0.3, bg=BG)
    L = ny * spacing[1]                            # every hitting ray crosses the slab along +y
    e = math.exp(-sig * L)
    want = np.concatenate([rgb * (1 - e) + np.array(BG[:3]) * e, [1 - e * (1 - BG[3])]])
    hit = np.abs(img[0] - np.array(BG)).max(axis=-1) > 0
    assert hit.sum() >= 5 * 7                      # the 9x7 view is wider than the box
    assert np.abs(img[0][hit] - want).max() < 1e-12
    # perspective: the centre pixel of view 0 looks along -x through the centre
    cams = synth.turntable_cameras(nx, ny, nz, spacing, n_views=1)
    img, _ = R.render(vol, spacing, _const_tf(rgb, sig), cams, 5, 5, 0.3, bg=BG)
    e = math.exp(-sig * nx * spacing[0])
    want = np.concatenate([rgb * (1 - e) + np.array(BG[:3]) * e, [1 - e * (1 - BG[3])]])
    assert np.abs(img[0, 2, 2] - want).max() < 1e-12


def _axis_camera(axis, nx, ny, nz, sp):
    """Orthographic view marching along +axis (0 = x, 1 = y, 2 = z)."""
    ext = np.array([nx, ny, nz], float) * np.array(sp, float)
    c = ext / 2
    cam = np.zeros((1, 11))
    d = np.zeros(3)
    d[axis] = 1.0
    cam[0, 0:3] = c - 3 * ext.max() * d
    cam[0, 3:6] = c
    cam[0, 6:9] = (0, 0, 1) if axis != 2 else (0, 1, 0)
    cam[0, 10] = ext.max()
    return cam


@pytest.mark.parametrize("axis,sp,step", [(0, (1, 1, 1), 0.5), (1, (1, 1.5, 1), 0.75),
                                          (2, (1, 1, 0.5), 0.25), (1, (1, 1, 1), 1.0)])
def test_linear_ramp_midpoint_exact(axis, sp, step):
    # density linear in the voxel index along one axis, sigma linear in s:
    # tau = c * g * s_axis * n_axis^2 / 2 (clamped half-voxels at both faces).
    n = [5, 6, 7]
    g = 1.0 / (n[axis] + 1)
    idx = np.indices((n[2], n[1], n[0]))[2 - axis].astype(np.float64)
    vol = g * (idx + 0.5)
    c = 0.8
    rgb = np.array([0.3, 0.6, 0.9])
    cam = _axis_camera(axis, *n, sp)
    img, _ = R.render(vol, sp, _linear_tf(rgb, c), cam, 4, 4, step, bg=BG)
    tau = c * g * sp[axis] * n[axis] ** 2 / 2.0
    e = math.exp(-tau)
    want = np.concatenate([rgb * (1 - e) + np.array(BG[:3]) * e, [1 - e * (1 - BG[3])]])
    inside = img[0][np.abs(img[0] - np.array(BG)).max(axis=-1) > 0]
    assert len(inside) > 0
    assert np.abs(inside - want).max() < 1e-12


def test_density_is_tent_sum_single_voxel():
    nx, ny, nz = 7, 6, 5
    sp = (1.0, 2.0, 0.5)
    vol = np.zeros((nz, ny, nx))
    v = (3, 2, 2)                                  # (x, y, z) interior voxel
    vol[v[2], v[1], v[0]] = 0.8
    rng = np.random.default_rng(7)
    q = rng.uniform(1.0, np.array([nx, ny, nz]) - 1.0, size=(400, 3))   # index space
    pts = q * np.array(sp)
    got = R.density_at(vol, sp, pts)
    tent = 0.8 * np.prod(np.maximum(0.0, 1.0 - np.abs(q - (np.array(v) + 0.5))), axis=1)
    assert np.abs(got - tent).max() < 1e-14


def test_single_voxel_render_brute_force():
    nx, ny, nz = 8, 7, 9
    sp = (1.0, 1.0, 1.0)
    vol = np.zeros((nz, ny, nx))
    vx = (4, 3, 5)
    vol[vx[2], vx[1], vx[0]] = 0.9
    tf = _linear_tf(np.array([0.9, 0.5, 0.2]), 2.0)
    cams = synth.turntable_cameras(nx, ny, nz, sp, n_views=3)
    W, H, step = 24, 20, 0.5
    o, d = RT.rays(cams, W, H)
    pix = np.array([(v, j, i) for v in range(3) for j in range(H) for i in range(W)])
    got, _ = R.render_pixels(vol, sp, tf, cams, W, H, step, pix, bg=BG)
    ext = np.array([nx, ny, nz], float)
    checked = 0
    for k in range(len(pix)):
        tin, tout = 0.0, np.inf
        ok = True
        for a in range(3):
            if d[k, a] == 0:
                ok &= 0 <= o[k, a] <= ext[a]
                continue
            t1, t2 = (0 - o[k, a]) / d[k, a], (ext[a] - o[k, a]) / d[k, a]
            tin, tout = max(tin, min(t1, t2)), min(tout, max(t1, t2))
        if not ok or tout <= tin:
            assert (got[k] == np.array(BG)).all()
            continue
        L = tout - tin
        n = max(1, math.ceil(L / step))
        T, Cc = 1.0, np.zeros(3)
        for i in range(n):
            ln = step if i < n - 1 else L - (n - 1) * step
            p = o[k] + (tin + i * step + ln / 2) * d[k]
            s = 0.9 * np.prod(np.maximum(0.0, 1.0 - np.abs(p - (np.array(vx) + 0.5))))
            sig = 2.0 * s
            e = math.exp(-sig * ln)
            Cc += T * (1 - e) * tf[0, :3]
            T *= e
        want = np.concatenate([Cc + T * np.array(BG[:3]), [1 - T * (1 - BG[3])]])
        assert np.abs(got[k] - want).max() < 1e-12
        checked += T < 1.0
    assert checked > 20                            # some rays do see the voxel


def test_quarter_turn_symmetry_sphere():
    n = 12
    idx = np.indices((n, n, n)).astype(float) + 0.5
    r = np.sqrt(((idx - n / 2) ** 2).sum(axis=0))
    vol = np.clip(1.0 - r / 5.0, 0.0, 1.0) * 0.6
    cams = synth.turntable_cameras(n, n, n, n_views=4)
    img, _ = R.render(vol, (1, 1, 1), synth.default_tf(sigma_scale=4.0), cams, 20, 20, 0.5, bg=BG)
    assert img[0].std() > 1e-3
    for v in range(1, 4):
        assert np.abs(img[v] - img[0]).max() < 1e-9


def test_mirror_x():
    rng = np.random.default_rng(8)
    vol = rng.uniform(0, 0.6, size=(6, 5, 7))
    cam = synth.front_ortho_camera(7, 5, 6)
    tf = synth.default_tf(sigma_scale=3.0)
    a, _ = R.render(vol, (1, 1, 1), tf, cam, 14, 12, 0.5)
    b, _ = R.render(vol[:, :, ::-1].copy(), (1, 1, 1), tf, cam, 14, 12, 0.5)
    assert np.abs(a[0][:, ::-1] - b[0]).max() < 1e-12


def test_orientation_of_image_axes():
    # ortho view along +y with up = +z: column grows with x, row 0 is the top (high z)
    nx, ny, nz = 4, 6, 8
    vol = np.zeros((nz, ny, nx))
    vol[5, 2, 1] = 1.0
    cam = synth.front_ortho_camera(nx, ny, nz)
    img, _ = R.render(vol, (1, 1, 1), _linear_tf(np.ones(3), 5.0), cam, 8, 8, 0.25)
    j, i = np.unravel_index(np.argmax(img[0, :, :, 3]), (8, 8))
    h = 0.5 * max(nx, nz)
    x_world, z_world = 1.5, 5.5
    i_want = ((x_world - nx / 2) / h + 1) * 8 / 2 - 0.5
    j_want = (1 - (z_world - nz / 2) / h) * 8 / 2 - 0.5
    assert abs(i - i_want) <= 0.5 and abs(j - j_want) <= 0.5


def test_step_refinement_second_order():
    n = 16
    idx = np.indices((n, n, n)).astype(float) + 0.5
    vol = 0.7 * np.exp(-(((idx - 8.0) ** 2).sum(axis=0)) / 18.0)
    tf = _linear_tf(np.array([0.5, 0.7, 0.9]), 1.5)
    cams = synth.turntable_cameras(n, n, n, n_views=2)
    ref, _ = R.render(vol, (1, 1, 1), tf, cams, 16, 16, 1.0 / 64)
    errs = []
    for st in (1.0, 0.5, 0.25):
        img, _ = R.render(vol, (1, 1, 1), tf, cams, 16, 16, st)
        errs.append(np.abs(img - ref).max())
    assert 2.5 < errs[0] / errs[1] < 6 and 2.5 < errs[1] / errs[2] < 6


def test_sample_count():
    vol = np.zeros((64, 64, 64), dtype=np.uint16)
    cam = synth.front_ortho_camera(64, 64, 64)
    _, cnt = R.render(vol, (1, 1, 1), synth.default_tf(), cam, 32, 32, 0.5)
    assert cnt[0] == 32 * 32 * 128                  # every ray crosses 64 voxels
    # opaque medium: T_i = exp(-sigma * 0.5 * i) >= 2^-14 for i <= 14 ln2 / (0.5 sigma)
    vol[:] = 65535
    sig = 2.0
    _, cnt = R.render(vol, (1, 1, 1), _const_tf(0.5, sig), cam, 32, 32, 0.5)
    per_ray = math.floor(14 * math.log(2) / (0.5 * sig)) + 1
    assert cnt[0] == 32 * 32 * per_ray


def _front_march_brute(vol, sp, tf, cam, W, H, step, ert_eps):
    """Hand-written march of the orthographic front view (rays along +y):
    every hitting ray has L = ny * spacing_y exactly, n = ceil(L / step)."""
    nz, ny, nx = vol.shape
    o, d = RT.rays(cam, W, H)
    L = ny * sp[1]
    n = max(1, math.ceil(L / step))
    out, counts = [], []
    for k in range(len(o)):
        x, z = o[k, 0], o[k, 2]
        if not (0 <= x <= nx * sp[0] and 0 <= z <= nz * sp[2]):
            out.append(np.array(BG))
            counts.append(0)
            continue
        T, Cc, cnt = 1.0, np.zeros(3), 0
        for i in range(n):
            ln = step if i < n - 1 else L - (n - 1) * step
            y = (i * step + 0.5 * ln) / sp[1] - 0.5          # voxel coordinate along y
            s = R.density_at(vol, sp, [[x, (y + 0.5) * sp[1], z]])[0]
            xx = min(max(s, 0.0), 1.0) * 255.0
            kk = min(int(math.floor(xx)), 254)
            w = xx - kk
            q = (1 - w) * tf[kk] + w * tf[kk + 1]
            e = math.exp(-q[3] * ln)
            cnt += T >= ert_eps
            Cc += T * (1 - e) * q[:3]
            T *= e
        out.append(np.concatenate([Cc + T * np.array(BG[:3]), [1 - T * (1 - BG[3])]]))
        counts.append(cnt)
    return np.array(out).reshape(H, W, 4), np.array(counts)


@pytest.mark.parametrize("step,n_want", [(0.5, 20), (0.5 * (1 - 2.0 ** -20), 21)])
def test_exact_multiple_step_count(step, n_want):
    """A segment that is a whole number of steps (L = 10 along +y, step 0.5)
    takes exactly L/step samples; a step a hair shorter gives ceil(L/step) =
    L/step + 1 samples, the last a sliver of length L - 20 step."""
    rng = np.random.default_rng(31)
    nx, ny, nz = 5, 10, 6
    vol = rng.uniform(0.0, 0.4, size=(nz, ny, nx))
    tf = _linear_tf(np.array([0.8, 0.3, 0.6]), 0.7)
    cam = synth.front_ortho_camera(nx, ny, nz)
    W, H = 6, 5
    img, cnt = R.render(vol, (1, 1, 1), tf, cam, W, H, step, ert_eps=0.0, bg=BG)
    ref, per_ray = _front_march_brute(vol, (1, 1, 1), tf, cam, W, H, step, 0.0)
    assert np.abs(img[0] - ref).max() < 1e-13
    hit = per_ray > 0
    assert hit.sum() >= 20 and (per_ray[hit] == n_want).all()
    assert cnt[0] == per_ray.sum()


def test_count_bounds_at_exact_multiples():
    """On rays whose length is exactly 128 steps, a lower-precision length may
    round up: hi allows the one extra sliver step, lo does not.  A step a hair
    shorter (129 samples, the last a sliver) gives the opposite bounds."""
    vol = np.zeros((64, 64, 64), dtype=np.uint16)
    cam = synth.front_ortho_camera(64, 64, 64)
    rays = 32 * 32
    _, cnt, b = R.render(vol, (1, 1, 1), synth.default_tf(), cam, 32, 32, 0.5, bounds=True)
    assert cnt[0] == rays * 128 and b[0, 0] == rays * 128 and b[0, 1] == rays * 129
    _, cnt, b = R.render(vol, (1, 1, 1), synth.default_tf(), cam, 32, 32, 0.5 * (1 - 2.0 ** -20),
                         bounds=True)
    assert cnt[0] == rays * 129 and b[0, 0] == rays * 128 and b[0, 1] == rays * 129
    # a step count far from a whole number: the bounds close on the count
    _, cnt, b = R.render(vol, (1, 1, 1), synth.default_tf(), cam, 32, 32, 0.3, bounds=True)
    assert cnt[0] == rays * 214 and b[0, 0] == b[0, 1] == cnt[0]


def test_count_bounds_at_the_termination_threshold():
    """Opaque medium, step 0.5, T_k = exp(-0.5 sigma k).  With sigma = 2 ln 2,
    T_14 = 2^-14 up to rounding: the sample at which T falls below the
    threshold is ambiguous, so [lo, hi] = [14, 15] per ray.  With sigma = 2 no
    T_k lies near 2^-14 and the bounds close on the count of 1 + floor(14 ln 2)."""
    vol = np.full((64, 64, 64), 65535, dtype=np.uint16)
    cam = synth.front_ortho_camera(64, 64, 64)
    rays = 32 * 32
    _, cnt, b = R.render(vol, (1, 1, 1), _const_tf(0.5, 2.0 * math.log(2.0)), cam, 32, 32, 0.5,
                         bounds=True)
    assert b[0, 0] == rays * 14 and b[0, 1] == rays * 15
    assert b[0, 0] <= cnt[0] <= b[0, 1]
    _, cnt, b = R.render(vol, (1, 1, 1), _const_tf(0.5, 2.0), cam, 32, 32, 0.5, bounds=True)
    per_ray = math.floor(14 * math.log(2)) + 1
    assert cnt[0] == b[0, 0] == b[0, 1] == rays * per_ray


def test_count_bounds_bracket_per_pixel():
    """Per-pixel counts of a turntable scene lie within their own bounds, and
    the bounds are at most one sample either side for each decision."""
    rng = np.random.default_rng(4)
    vol = rng.integers(0, 40000, size=(12, 10, 14)).astype(np.uint16)
    cams = synth.turntable_cameras(14, 10, 12, n_views=4)
    pix = np.array([(v, j, i) for v in range(4) for j in range(9) for i in range(11)])
    _, tot, c = R.render_pixels(vol, (1, 1, 1), synth.default_tf(sigma_scale=8.0), cams, 11, 9, 0.5,
                                pix, per_pixel=True)
    assert (c[:, 1] <= c[:, 0]).all() and (c[:, 0] <= c[:, 2]).all()
    assert (c[:, 0] - c[:, 1] <= 2).all() and (c[:, 2] - c[:, 0] <= 2).all()
    assert tot == c[:, 0].sum()


def test_torch_twin_matches_c_oracle():
    rng = np.random.default_rng(9)
    d = rng.uniform(0, 0.6, size=(11, 9, 10))
    sp = (1.0, 1.3, 0.7)
    tf = synth.random_tf(10).astype(np.float64)
    cams = np.concatenate([synth.turntable_cameras(10, 9, 11, sp, n_views=3),
                           synth.front_ortho_camera(10, 9, 11, sp)])
    a, _ = R.render(d, sp, tf, cams, 13, 11, 0.4, ert_eps=0.0, bg=BG)
    b = RT.render(torch.tensor(d), torch.tensor(tf), cams, 13, 11, 0.4, sp, bg=BG).numpy()
    assert np.abs(a - b).max() < 1e-13


def test_torch_twin_gradient_matches_finite_differences():
    rng = np.random.default_rng(11)
    d = rng.uniform(0.05, 0.5, size=(8, 8, 8))
    tf = synth.random_tf(12).astype(np.float64)
    cams = synth.turntable_cameras(8, 8, 8, n_views=2)
    tgt = rng.uniform(0, 1, size=(2, 10, 10, 4))
    dt = torch.tensor(d, requires_grad=True)
    tt = torch.tensor(tf, requires_grad=True)
    loss = ((RT.render(dt, tt, cams, 10, 10, 0.5) - torch.tensor(tgt)) ** 2).mean()
    loss.backward()

    def L(dd, ff):
        img, _ = R.render(dd, (1, 1, 1), ff, cams, 10, 10, 0.5, ert_eps=0.0)
        return ((img - tgt) ** 2).mean()

    h = 1e-6
    for _ in range(8):
        z, y, x = rng.integers(1, 7, size=3)
        dp, dm = d.copy(), d.copy()
        dp[z, y, x] += h
        dm[z, y, x] -= h
        fd = (L(dp, tf) - L(dm, tf)) / (2 * h)
        assert abs(fd - dt.grad[z, y, x].item()) < 1e-6 * max(1.0, abs(fd)) + 1e-9
    for _ in range(8):
        k, c = int(rng.integers(0, 256)), int(rng.integers(0, 4))
        fp, fm = tf.copy(), tf.copy()
        fp[k, c] += h
        fm[k, c] -= h
        fd = (L(d, fp) - L(d, fm)) / (2 * h)
        assert abs(fd - tt.grad[k, c].item()) < 1e-6 * max(1.0, abs(fd)) + 1e-9


def test_torch_twin_gradient_analytic_single_material():
    """A box of constant density s seen along +y, a TF of constant colour and
    sigma(s) = c s: the pixel is Beer-Lambert, I = rgb (1 - e) + bg e with
    e = exp(-c s L), whatever the sampling.  Closed-form gradients: the summed
    density gradient is dI/ds = (rgb - bg) c L e; the two TF knots around s
    carry (1 - w) and w of dI/dsigma = (rgb - bg) L e (w = 255 s - k), the
    colour knots (1 - w) and w of dI/drgb = 1 - e."""
    nx, ny, nz = 4, 6, 5
    s0, c = 0.3, 0.9
    rgb = np.array([0.7, 0.2, 0.4])
    L = float(ny)
    dens = torch.full((nz, ny, nx), s0, dtype=torch.float64, requires_grad=True)
    tf = torch.tensor(_linear_tf(rgb, c), dtype=torch.float64, requires_grad=True)
    cam = synth.front_ortho_camera(nx, ny, nz)
    img = RT.render(dens, tf, cam, 9, 7, 0.35, bg=BG)
    hit = (img[0] - torch.tensor(BG, dtype=torch.float64)).abs().amax(dim=-1) > 0
    pix = hit.nonzero()[len(hit.nonzero()) // 2]
    I = img[0, pix[0], pix[1], 0]                  # red channel of one hitting pixel
    I.backward()
    e = math.exp(-c * s0 * L)
    assert abs(I.item() - (rgb[0] * (1 - e) + BG[0] * e)) < 1e-13
    assert abs(dens.grad.sum().item() - (rgb[0] - BG[0]) * c * L * e) < 1e-12
    k = int(255 * s0)
    w = 255 * s0 - k
    g_sigma = (rgb[0] - BG[0]) * L * e
    assert abs(tf.grad[k, 3].item() - (1 - w) * g_sigma) < 1e-12
    assert abs(tf.grad[k + 1, 3].item() - w * g_sigma) < 1e-12
    assert abs(tf.grad[k, 0].item() - (1 - w) * (1 - e)) < 1e-12
    assert abs(tf.grad[k + 1, 0].item() - w * (1 - e)) < 1e-12
    others = torch.ones(256, dtype=torch.bool)
    others[k] = others[k + 1] = False
    assert tf.grad[others].abs().max().item() == 0.0


def _pix(V, H, W, K, seed):
    rng = np.random.default_rng(seed)
    return np.stack([rng.integers(0, V, K), rng.integers(0, H, K), rng.integers(0, W, K)], axis=1)


def test_march_rays_matches_both_oracles():
    """The per-ray form of the torch twin against the C oracle and the step-by-step
    twin, on sampled pixels of perspective and orthographic views (misses included)."""
    rng = np.random.default_rng(21)
    d = rng.uniform(0, 0.6, size=(11, 9, 10))
    sp = (1.0, 1.3, 0.7)
    tf = synth.random_tf(22).astype(np.float64)
    cams = np.concatenate([synth.turntable_cameras(10, 9, 11, sp, n_views=3),
                           synth.front_ortho_camera(10, 9, 11, sp)])
    W, H = 13, 11
    pix = np.concatenate([_pix(4, H, W, 60, 23), [[3, 0, 0], [0, 5, 6]]])
    o, dd = RT.pixel_rays(cams, W, H, pix)
    got = RT.march_rays(torch.tensor(d), torch.tensor(tf), o, dd, 0.4, sp, bg=BG).numpy()
    ref_c, _ = R.render_pixels(d, sp, tf, cams, W, H, 0.4, pix, ert_eps=0.0, bg=BG)
    full = RT.render(torch.tensor(d), torch.tensor(tf), cams, W, H, 0.4, sp, bg=BG).numpy()
    assert np.abs(got - ref_c).max() < 1e-13
    assert np.abs(got - full[pix[:, 0], pix[:, 1], pix[:, 2]]).max() < 1e-13
    assert (np.abs(got - np.array(BG)).max(axis=1) > 0.01).sum() > 15     # a third of them show the volume


def test_march_rays_beer_lambert():
    nx, ny, nz = 6, 10, 8
    vol = torch.full((nz, ny, nx), 20000 / 65535, dtype=torch.float64)
    rgb, sig = np.array([0.7, 0.2, 0.4]), 0.13
    cam = synth.front_ortho_camera(nx, ny, nz)
    o, d = RT.pixel_rays(cam, 9, 7, [[0, 3, 4]])                 # the centre pixel
    got = RT.march_rays(vol, torch.tensor(_const_tf(rgb, sig)), o, d, 0.3, bg=BG).numpy()[0]
    e = math.exp(-sig * ny)
    want = np.concatenate([rgb * (1 - e) + np.array(BG[:3]) * e, [1 - e * (1 - BG[3])]])
    assert np.abs(got - want).max() < 1e-12


def test_march_rays_gradient_matches_step_by_step_twin():
    rng = np.random.default_rng(24)
    d = rng.uniform(0.05, 0.5, size=(8, 9, 7))
    tf = synth.random_tf(25).astype(np.float64)
    cams = synth.turntable_cameras(7, 9, 8, n_views=2)
    W = H = 10
    pix = _pix(2, H, W, 40, 26)
    wts = torch.tensor(rng.uniform(-1, 1, size=(len(pix), 4)))
    d1, t1 = torch.tensor(d, requires_grad=True), torch.tensor(tf, requires_grad=True)
    o, dd = RT.pixel_rays(cams, W, H, pix)
    (RT.march_rays(d1, t1, o, dd, 0.5) * wts).sum().backward()
    d2, t2 = torch.tensor(d, requires_grad=True), torch.tensor(tf, requires_grad=True)
    img = RT.render(d2, t2, cams, W, H, 0.5)
    (img[pix[:, 0], pix[:, 1], pix[:, 2]] * wts).sum().backward()
    assert d1.grad.abs().max() > 0 and t1.grad.abs().max() > 0
    assert (d1.grad - d2.grad).abs().max() < 1e-12
    assert (t1.grad - t2.grad).abs().max() < 1e-12
