"""GPU parity of the ray caster against the FP64 oracle: max-abs <= 2e-4 on RGBA."""
import math

import numpy as np
import pytest
import torch

from oracle import reduce as O
from oracle import render as R
from paper_2311_15038_amd import synth
from paper_2311_15038_amd import vr

from gpu_util import banner, dev, to_dev_u16

pytestmark = pytest.mark.gpu

TOL = 2e-4
BG = (0.25, 0.5, 0.125, 0.75)


@pytest.fixture(scope="module")
def level1(small_volume):
    H, Ht = O.histogram(small_volume), O.histogram(small_volume, 0, 3)
    return O.pyramid(small_volume, O.keep_bits(O.valley_threshold(H), Ht), 1)[0]


def _tf_dev(tf):
    return torch.from_numpy(np.ascontiguousarray(tf, dtype=np.float32)).to(dev())


def test_small_config_front_view(level1):
    """64^3 level, one 256 x 256 orthographic view, step 0.5, default TF."""
    banner("raycast 64^3 ortho 256^2")
    tf = synth.default_tf()
    cam = synth.front_ortho_camera(64, 64, 64)
    cnt = torch.zeros(2, dtype=torch.int64, device=dev())
    img = vr.vr_raycast(to_dev_u16(level1), _tf_dev(tf), cam, 256, 256, 0.5, samples=cnt)
    ref, n_ref, lohi = R.render(level1, (1, 1, 1), tf.astype(np.float64), cam, 256, 256, 0.5,
                                bounds=True)
    err = np.abs(img.cpu().numpy() - ref).max()
    assert err <= TOL, err
    assert ref[..., 3].max() > 0.5                        # the view does show the specimen
    n_gpu = int(cnt[0].item())
    assert int(cnt[1].item()) == n_gpu               # no occupancy: every sample evaluated
    # every ray crosses the box along +y with L = 64 exactly: 128 steps on both sides (the
    # oracle's upper bound allows a 129th on each ray, since L/step is an integer) and no
    # ray's transmittance comes near 2^-14, so the count is the oracle's exactly
    lo, hi = int(lohi[0, 0]), int(lohi[0, 1])
    assert lo == 256 * 256 * 128 and hi == 256 * 256 * 129, (lo, hi)
    assert n_gpu == int(n_ref[0]) == lo, (n_gpu, int(n_ref[0]))


def test_turntable_perspective(level1):
    banner("raycast 64^3 turntable 36 x 48^2")
    tf = synth.default_tf(sigma_scale=2.0)
    cams = synth.turntable_cameras(64, 64, 64, n_views=36)
    img = vr.vr_raycast(to_dev_u16(level1), _tf_dev(tf), cams, 48, 48, 0.5, bg=BG)
    ref, _ = R.render(level1, (1, 1, 1), tf.astype(np.float64), cams, 48, 48, 0.5, bg=BG)
    assert np.abs(img.cpu().numpy() - ref).max() <= TOL


def test_many_views_split_launches(level1):
    banner("raycast 50 views (two launches)")
    tf = synth.default_tf()
    cams = synth.turntable_cameras(64, 64, 64, n_views=50)
    img = vr.vr_raycast(to_dev_u16(level1), _tf_dev(tf), cams, 20, 16, 0.75)
    ref, _ = R.render(level1, (1, 1, 1), tf.astype(np.float64), cams, 20, 16, 0.75)
    assert np.abs(img.cpu().numpy() - ref).max() <= TOL


@pytest.mark.parametrize("W,H", [(37, 23), (1, 1), (16, 48)])
def test_f32_anisotropic_ragged(W, H):
    banner(f"raycast f32 anisotropic {W}x{H}")
    rng = np.random.default_rng(21)
    nz, ny, nx = 25, 30, 20
    idx = np.indices((nz, ny, nx)).astype(np.float64)
    vol = 0.3 + 0.25 * np.sin(idx[0] / 3.0) * np.cos(idx[1] / 4.0) + 0.05 * rng.random((nz, ny, nx))
    vol = vol.astype(np.float32)
    sp = (1.0, 0.7, 1.3)
    tf = synth.random_tf(22, sigma_max=0.4)
    cams = np.concatenate([synth.turntable_cameras(nx, ny, nz, sp, n_views=5),
                           synth.front_ortho_camera(nx, ny, nz, sp)])
    img = vr.vr_raycast(torch.from_numpy(vol).to(dev()), _tf_dev(tf), cams, W, H, 0.4, sp, bg=BG)
    ref, _ = R.render(vol, sp, tf.astype(np.float64), cams, W, H, 0.4, bg=BG)
    assert np.abs(img.cpu().numpy() - ref).max() <= TOL


def test_no_early_termination(level1):
    banner("raycast ERT off")
    tf = synth.default_tf(sigma_scale=4.0)
    cams = synth.turntable_cameras(64, 64, 64, n_views=3)
    img = vr.vr_raycast(to_dev_u16(level1), _tf_dev(tf), cams, 40, 40, 0.5, ert_eps=0.0)
    ref, _ = R.render(level1, (1, 1, 1), tf.astype(np.float64), cams, 40, 40, 0.5, ert_eps=0.0)
    assert np.abs(img.cpu().numpy() - ref).max() <= TOL


def test_empty_volume_background_exact():
    banner("raycast empty volume")
    vol = torch.zeros((9, 7, 5), dtype=torch.uint16, device=dev())
    cams = np.concatenate([synth.turntable_cameras(5, 7, 9, n_views=3),
                           synth.front_ortho_camera(5, 7, 9)])
    img = vr.vr_raycast(vol, _tf_dev(synth.default_tf()), cams, 16, 12, 0.5, bg=BG)
    assert (img.cpu().numpy() == np.array(BG, dtype=np.float32)).all()


def test_constant_slab_beer_lambert():
    banner("raycast constant slab")
    nx, ny, nz = 6, 10, 8
    vol = torch.full((nz, ny, nx), 20000, dtype=torch.int32).to(torch.uint16).to(dev())
    tf = np.zeros((256, 4), np.float32)
    tf[:, :3] = (0.7, 0.2, 0.4)
    tf[:, 3] = 0.13
    cam = synth.front_ortho_camera(nx, ny, nz)
    img = vr.vr_raycast(vol, _tf_dev(tf), cam, 9, 7, 0.3, bg=BG).cpu().numpy()[0]
    e = math.exp(-0.13 * ny)
    want = np.array([0.7 * (1 - e) + BG[0] * e, 0.2 * (1 - e) + BG[1] * e,
                     0.4 * (1 - e) + BG[2] * e, 1 - e * (1 - BG[3])])
    hit = np.abs(img - np.array(BG)).max(axis=-1) > 0
    assert hit.sum() >= 35
    assert np.abs(img[hit] - want).max() <= 1e-5


def test_raycast_rejects_bad_args(level1):
    v = to_dev_u16(level1)
    tf = _tf_dev(synth.default_tf())
    cam = synth.front_ortho_camera(64, 64, 64)
    with pytest.raises(vr.VrError):
        vr.vr_raycast(v, tf, cam, 8, 8, 0.0)
    bad = synth.turntable_cameras(64, 64, 64, n_views=1)
    bad[0, 9] = 180.0
    with pytest.raises(vr.VrError):
        vr.vr_raycast(v, tf, bad, 8, 8, 0.5)
    with pytest.raises(vr.VrError):
        vr.vr_raycast(v, tf, cam, 0, 8, 0.5)


# ------------------------------------------------------------ brick render layout
def _apron(nbx, nby, elems_per_brick, dtype):
    """The zeros after the last brick: one brick layer, one brick row and one brick."""
    return np.zeros((nbx * nby + nbx + 1) * elems_per_brick, dtype=dtype)


def _brick_ref(a, e=4):
    """The brick layout (bricks of e^3 voxels, then the apron of zeros) and the dilated
    occupancy, written out with NumPy."""
    nz, ny, nx = a.shape
    nbz, nby, nbx = (nz + e - 1) // e, (ny + e - 1) // e, (nx + e - 1) // e
    pad = np.zeros((nbz * e, nby * e, nbx * e), dtype=a.dtype)
    pad[:nz, :ny, :nx] = a
    br = pad.reshape(nbz, e, nby, e, nbx, e).transpose(0, 2, 4, 1, 3, 5).reshape(-1)
    br = np.concatenate([br, _apron(nbx, nby, e ** 3, a.dtype)])
    occ = np.zeros((nbz, nby, nbx), dtype=np.uint8)
    for z, y, x in np.argwhere(a != 0):
        for zz in (z - 1, z):
            for yy in (y - 1, y):
                for xx in (x - 1, x):
                    if zz >= 0 and yy >= 0 and xx >= 0:
                        occ[zz // e, yy // e, xx // e] = 1
    mz, my, mx = (nbz + 3) // 4, (nby + 3) // 4, (nbx + 3) // 4
    pad = np.zeros((mz * 4, my * 4, mx * 4), dtype=np.uint8)
    pad[:nbz, :nby, :nbx] = occ
    macro = pad.reshape(mz, 4, my, 4, mx, 4).max(axis=(1, 3, 5))
    # Chebyshev distance over bricks to the nearest marked brick, capped (brute force)
    cap = vr.BRICK_DIST_CAP
    marked = np.argwhere(occ != 0)
    grid = np.indices(occ.shape).reshape(3, -1).T
    if len(marked):
        dist = np.abs(grid[:, None, :] - marked[None, :, :]).max(axis=2).min(axis=1)
    else:
        dist = np.full(len(grid), cap)
    dist = np.minimum(dist, cap).astype(np.uint8)
    return br, np.concatenate([occ.reshape(-1), macro.reshape(-1), dist])


def _occ_parts(occ_t, shape, layout=vr.LAYOUT_BRICK4):
    """The marks, group marks and distance grid of an occupancy tensor (the working
    bytes after them are left out)."""
    nz, ny, nx = shape
    nb, _, nocc = vr.vr_brick_count_layout(layout, nx, ny, nz)
    assert occ_t.numel() == nocc
    return occ_t.cpu().numpy()[:nocc - nb]


# nx a multiple of 4 takes whole-row vector loads: (8, 8, 8), (7, 5, 12), (13, 30, 64)
@pytest.mark.parametrize("shape", [(8, 8, 8), (9, 6, 13), (1, 1, 1), (29, 23, 37), (70, 33, 81), (7, 5, 12),
                                   (13, 30, 64)])
def test_brick_layout_and_occupancy(shape):
    banner(f"brick layout {shape}")
    rng = np.random.default_rng(31)
    a = np.zeros(shape, dtype=np.uint16)
    m = rng.random(shape) < 0.01
    a[m] = rng.integers(1, 65536, size=int(m.sum()))
    a[0, 0, 0] = 7
    a[-1, -1, -1] = 9
    bv = vr.vr_brick_volume(to_dev_u16(a))
    br, occ = _brick_ref(a)
    got = bv.data.cpu().view(torch.int16).numpy().view(np.uint16)
    assert (got == br).all()
    assert (_occ_parts(bv.occupancy, shape) == occ).all()
    f = a.astype(np.float32) / 7.0
    bf = vr.vr_brick_volume(torch.from_numpy(f).to(dev()))
    assert (bf.data.cpu().numpy() == _brick_ref(f)[0]).all()
    assert (_occ_parts(bf.occupancy, shape) == occ).all()


@pytest.mark.parametrize("shape", [(40, 36, 120), (9, 70, 33)])
def test_brick_distance_grid_far_from_anything(shape):
    """Two non-zero voxels in a large empty volume: distances from 0 up to the cap,
    against brute force (and an empty volume, all at the cap)."""
    banner(f"brick distance grid {shape}")
    a = np.zeros(shape, dtype=np.uint16)
    a[1, 2, 3] = 500
    a[-2, -3, -5] = 65535
    bv = vr.vr_brick_volume(to_dev_u16(a))
    ref = _brick_ref(a)[1]
    got = _occ_parts(bv.occupancy, shape)
    assert (got == ref).all()
    nb = vr.vr_brick_count(*shape[::-1])[0]
    assert got[-nb:].max() == vr.BRICK_DIST_CAP and (got[-nb:] == 0).sum() >= 2
    e = vr.vr_brick_volume(to_dev_u16(np.zeros(shape, dtype=np.uint16)))
    assert (_occ_parts(e.occupancy, shape)[-nb:] == vr.BRICK_DIST_CAP).all()


@pytest.mark.parametrize("shape", [(8, 8, 8), (9, 6, 13), (1, 1, 1), (29, 23, 37), (17, 40, 70)])
def test_brick8_layout_and_occupancy(shape):
    """8^3 bricks: layout, marks, group marks and distance grid against NumPy."""
    banner(f"brick8 layout {shape}")
    rng = np.random.default_rng(35)
    a = np.zeros(shape, dtype=np.uint16)
    m = rng.random(shape) < 0.005
    a[m] = rng.integers(1, 65536, size=int(m.sum()))
    a[0, 0, 0] = 7
    a[-1, -1, -1] = 9
    bv = vr.vr_brick_volume(to_dev_u16(a), edge=8)
    assert bv.layout == vr.LAYOUT_BRICK8
    br, occ = _brick_ref(a, 8)
    assert (bv.data.cpu().view(torch.int16).numpy().view(np.uint16) == br).all()
    assert (_occ_parts(bv.occupancy, shape, vr.LAYOUT_BRICK8) == occ).all()
    f = a.astype(np.float32) / 7.0
    bf = vr.vr_brick_volume(torch.from_numpy(f).to(dev()), edge=8)
    assert (bf.data.cpu().numpy() == _brick_ref(f, 8)[0]).all()
    assert (_occ_parts(bf.occupancy, shape, vr.LAYOUT_BRICK8) == occ).all()


def test_brick_layout_from_unaligned_source():
    """nx a multiple of 4 but the source one voxel past an aligned address: the voxel-by-voxel path."""
    banner("brick layout from an unaligned source")
    rng = np.random.default_rng(33)
    shape = (6, 9, 16)
    a = rng.integers(0, 65536, size=shape).astype(np.uint16)
    a[rng.random(shape) < 0.5] = 0
    flat = torch.zeros(a.size + 8, dtype=torch.int16, device=dev())
    flat[1:1 + a.size] = torch.from_numpy(a.reshape(-1).view(np.int16)).to(dev())
    src = flat[1:1 + a.size].view(shape)
    assert src.data_ptr() % 8 != 0
    bv = vr.vr_brick_volume(src)
    br, occ = _brick_ref(a)
    assert (bv.data.cpu().view(torch.int16).numpy().view(np.uint16) == br).all()
    assert (_occ_parts(bv.occupancy, shape) == occ).all()
    f = torch.zeros(a.size + 8, dtype=torch.float32, device=dev())
    f[2:2 + a.size] = torch.from_numpy(a.reshape(-1).astype(np.float32) / 5.0).to(dev())
    fs = f[2:2 + a.size].view(shape)
    assert fs.data_ptr() % 16 != 0
    bf = vr.vr_brick_volume(fs)
    assert (bf.data.cpu().numpy() == _brick_ref(a.astype(np.float32) / 5.0)[0]).all()


def _ovl_ref(a, pad_value=0):
    """The overlap layout (4^3 bricks, brick bx holding voxels 3 bx .. 3 bx + 3, then the
    apron) and its occupancy from the cells each brick serves, written out with NumPy."""
    nz, ny, nx = a.shape
    nbx, nby, nbz = (nx - 1) // 3 + 1, (ny + 3) // 4, (nz + 3) // 4
    pad = np.full((nbz * 4, nby * 4, 3 * nbx + 1), pad_value, dtype=a.dtype)
    pad[:nz, :ny, :nx] = a
    cols = np.stack([pad[:, :, 3 * np.arange(nbx) + e] for e in range(4)], axis=-1)   # [Z][Y][nbx][4]
    br = cols.reshape(nbz, 4, nby, 4, nbx, 4).transpose(0, 2, 4, 1, 3, 5).reshape(-1)
    br = np.concatenate([br, np.full((nbx * nby + nbx + 1) * 64, pad_value, dtype=a.dtype)])
    occ = np.zeros((nbz, nby, nbx), dtype=np.uint8)
    for z, y, x in np.argwhere(a != 0):
        # cells whose eight taps include (x, y, z): base taps x - {0, 1} (and likewise y, z)
        for zz in (z - 1, z):
            for yy in (y - 1, y):
                for xx in (x - 1, x):
                    if zz >= 0 and yy >= 0 and xx >= 0:
                        occ[zz // 4, yy // 4, xx // 3] = 1
    mz, my, mx = (nbz + 3) // 4, (nby + 3) // 4, (nbx + 3) // 4
    mpad = np.zeros((mz * 4, my * 4, mx * 4), dtype=np.uint8)
    mpad[:nbz, :nby, :nbx] = occ
    macro = mpad.reshape(mz, 4, my, 4, mx, 4).max(axis=(1, 3, 5))
    cap = vr.BRICK_DIST_CAP
    marked = np.argwhere(occ != 0)
    grid = np.indices(occ.shape).reshape(3, -1).T
    if len(marked):
        dist = np.abs(grid[:, None, :] - marked[None, :, :]).max(axis=2).min(axis=1)
    else:
        dist = np.full(len(grid), cap)
    dist = np.minimum(dist, cap).astype(np.uint8)
    return br, np.concatenate([occ.reshape(-1), macro.reshape(-1), dist])


@pytest.mark.parametrize("shape", [(8, 8, 8), (9, 6, 13), (1, 1, 1), (1, 1, 2), (3, 2, 3), (5, 7, 4),
                                   (29, 23, 37), (13, 30, 64)])
def test_overlap_layout_and_occupancy(shape):
    banner(f"overlap layout {shape}")
    rng = np.random.default_rng(33)
    a = np.zeros(shape, dtype=np.uint16)
    m = rng.random(shape) < 0.02
    a[m] = rng.integers(1, 65536, size=int(m.sum()))
    a[0, 0, 0] = 7
    a[-1, -1, -1] = 9
    bv = vr.vr_brick_volume(to_dev_u16(a), overlap=True)
    assert bv.layout == vr.LAYOUT_BRICK4_OVERLAP
    br, occ = _ovl_ref(a)
    got = bv.data.cpu().view(torch.int16).numpy().view(np.uint16)
    assert got.size == br.size and (got == br).all()
    assert (_occ_parts(bv.occupancy, shape, vr.LAYOUT_BRICK4_OVERLAP) == occ).all()
    # marks above a level: the occupancy of the volume with the voxels at or below it zeroed
    V = 30000
    bm = vr.vr_brick_volume(to_dev_u16(a), overlap=True, mark_above=V)
    assert (_occ_parts(bm.occupancy, shape, vr.LAYOUT_BRICK4_OVERLAP) == _ovl_ref(np.where(a > V, a, 0))[1]).all()
    with pytest.raises(vr.VrError):
        vr.vr_brick_volume(torch.from_numpy(a.astype(np.float32)).to(dev()), overlap=True)


@pytest.mark.parametrize("shape", [(64, 64, 64), (29, 23, 37), (40, 17, 50), (90, 70, 110), (16, 12, 5),
                                   (7, 9, 2), (6, 5, 1)])
def test_overlap_bit_identical(level1, shape):
    """Overlapping bricks (with the distance grid and TF-level marks) give the linear
    march's frames and taken counts bit for bit, on grazing and turntable views."""
    banner(f"overlap bricks == linear {shape}")
    a = level1 if shape == (64, 64, 64) else _sparse_volume(shape, 17)
    nz, ny, nx = a.shape
    tf_h = synth.default_tf(sigma_scale=3.0)
    tf = _tf_dev(tf_h)
    cams = np.concatenate([synth.turntable_cameras(nx, ny, nz, n_views=7),
                           synth.front_ortho_camera(nx, ny, nz), _grazing_cameras(nx, ny, nz)[::2]])
    v = to_dev_u16(a)
    c0 = torch.zeros(2, dtype=torch.int64, device=dev())
    lin = vr.vr_raycast(v, tf, cams, 45, 38, 0.5, samples=c0)
    for above in (0, vr.tf_mark_level(tf_h)):
        bo = vr.vr_brick_volume(v, overlap=True, mark_above=above)
        c1 = torch.zeros(2, dtype=torch.int64, device=dev())
        assert torch.equal(lin, vr.vr_raycast(bo, tf, cams, 45, 38, 0.5, samples=c1))
        assert c1[0].item() == c0[0].item() and c1[1].item() <= c1[0].item()
        bo.occupancy = None
        assert torch.equal(lin, vr.vr_raycast(bo, tf, cams, 45, 38, 0.5))
    if shape in ((29, 23, 37), (16, 12, 5)):
        # against the oracle on the turntable and orthographic views (rays exactly along
        # voxel boundaries, as in the grazing views, fall on either side in FP32 and FP64)
        ref, _ = R.render(a, (1, 1, 1), tf_h.astype(np.float64), cams[:8], 45, 38, 0.5)
        assert np.abs(lin[:8].cpu().numpy() - ref).max() <= TOL


def _pairs_ref(a):
    """The layout of x-tap pairs: element (x, y, z) = (a[z, y, x], a[z, y, min(x + 1, nx - 1)]),
    in brick order, as the interleaved low/high voxels."""
    nz, ny, nx = a.shape
    hi = np.concatenate([a[:, :, 1:], a[:, :, -1:]], axis=2)
    nbz, nby, nbx = (nz + 3) // 4, (ny + 3) // 4, (nx + 3) // 4
    pad = np.zeros((nbz * 4, nby * 4, nbx * 4, 2), dtype=a.dtype)
    pad[:nz, :ny, :nx, 0] = a
    pad[:nz, :ny, :nx, 1] = hi
    br = pad.reshape(nbz, 4, nby, 4, nbx, 4, 2).transpose(0, 2, 4, 1, 3, 5, 6).reshape(-1)
    return np.concatenate([br, _apron(nbx, nby, 128, a.dtype)])


@pytest.mark.parametrize("shape", [(8, 8, 8), (9, 6, 13), (1, 1, 1), (29, 23, 37), (5, 3, 4), (7, 5, 12)])
def test_pair_layout(shape):
    banner(f"pair layout {shape}")
    rng = np.random.default_rng(32)
    a = rng.integers(0, 65536, size=shape).astype(np.uint16)
    a[rng.random(shape) < 0.7] = 0
    bv = vr.vr_brick_volume(to_dev_u16(a), pairs=True)
    got = bv.data.cpu().view(torch.int16).numpy().view(np.uint16)
    assert (got == _pairs_ref(a)).all()
    assert (_occ_parts(bv.occupancy, shape) == _brick_ref(a)[1]).all()
    f = a.astype(np.float32) / 3.0
    bf = vr.vr_brick_volume(torch.from_numpy(f).to(dev()), pairs=True)
    assert (bf.data.cpu().numpy() == _pairs_ref(f)).all()


def _sparse_volume(shape, seed):
    """Blobs in empty space, some touching the faces: exercises brick skipping."""
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    idx = np.indices(shape).astype(np.float64)
    a = np.zeros(shape)
    for _ in range(6):
        c = rng.uniform(0, 1, 3) * np.array(shape)
        r = rng.uniform(2, 6)
        d2 = ((idx - c[:, None, None, None]) ** 2).sum(axis=0)
        a += 30000 * np.exp(-d2 / (2 * r * r)) * (d2 < 9 * r * r)
    return np.clip(a, 0, 65535).astype(np.uint16)


@pytest.mark.parametrize("shape", [(64, 64, 64), (29, 23, 37), (40, 17, 50), (90, 70, 110)])
def test_brick_and_skip_bit_identical(level1, shape):
    banner(f"bricked+skip == linear {shape}")
    a = level1 if shape == (64, 64, 64) else _sparse_volume(shape, 5)
    nz, ny, nx = a.shape
    tf = _tf_dev(synth.default_tf(sigma_scale=3.0))
    cams = np.concatenate([synth.turntable_cameras(nx, ny, nz, n_views=7),
                           synth.front_ortho_camera(nx, ny, nz)])
    v = to_dev_u16(a)
    c0 = torch.zeros(2, dtype=torch.int64, device=dev())
    c1 = torch.zeros(2, dtype=torch.int64, device=dev())
    c2 = torch.zeros(2, dtype=torch.int64, device=dev())
    lin = vr.vr_raycast(v, tf, cams, 45, 38, 0.5, samples=c0)
    bv = vr.vr_brick_volume(v)
    skip = vr.vr_raycast(bv, tf, cams, 45, 38, 0.5, samples=c1)
    bv.occupancy = None
    noskip = vr.vr_raycast(bv, tf, cams, 45, 38, 0.5, samples=c2)
    assert torch.equal(lin, noskip) and torch.equal(lin, skip)
    b8 = vr.vr_brick_volume(v, edge=8)
    c8 = torch.zeros(2, dtype=torch.int64, device=dev())
    assert torch.equal(lin, vr.vr_raycast(b8, tf, cams, 45, 38, 0.5, samples=c8))
    assert c8[0].item() == c0[0].item() and c8[1].item() <= c8[0].item()
    b8.occupancy = None
    assert torch.equal(lin, vr.vr_raycast(b8, tf, cams, 45, 38, 0.5))
    pv = vr.vr_brick_volume(v, pairs=True)
    c3 = torch.zeros(2, dtype=torch.int64, device=dev())
    assert torch.equal(lin, vr.vr_raycast(pv, tf, cams, 45, 38, 0.5, samples=c3))
    assert c3[0].item() == c0[0].item() and c3[1].item() == c1[1].item()
    pv.occupancy = None
    assert torch.equal(lin, vr.vr_raycast(pv, tf, cams, 45, 38, 0.5))
    assert c0[0].item() == c1[0].item() == c2[0].item()
    assert c0[1].item() == c0[0].item() and c2[1].item() == c2[0].item()
    assert c1[1].item() <= c1[0].item()               # skipped samples are counted, not evaluated
    if shape != (64, 64, 64):
        ref, n_ref, lohi = R.render(a, (1, 1, 1), synth.default_tf(sigma_scale=3.0).astype(np.float64),
                                    cams, 45, 38, 0.5, bounds=True)
        assert np.abs(skip.cpu().numpy() - ref).max() <= TOL
        # the count the skipping march reports (passed-over samples included) is the oracle's
        assert int(lohi[:, 0].sum()) <= c1[0].item() <= int(lohi[:, 1].sum()), (c1, n_ref.sum(), lohi.sum(0))


@pytest.mark.parametrize("shape,edge", [((64, 64, 64), 4), ((29, 23, 37), 4), ((32, 40, 48), 8), ((21, 30, 13), 8),
                                        ((64, 64, 64), 3), ((29, 23, 37), 3)])
def test_far_taps_past_the_volume_have_no_weight(shape, edge):
    """The u16 march reads the far taps of cells on the volume's last voxel layer from
    the bricks' padding, the next brick, brick row or layer, or the apron after the last
    brick, with weight 0: filling all of those with 65535 leaves the frames equal to the
    linear march's bit for bit."""
    banner(f"far taps past the volume {shape} bricks {edge}")
    a = _sparse_volume(shape, 13)
    a[0, :, :] = 20000            # faces with content, so that rays sample the last layers
    a[:, -1, :] = 30000
    a[:, :, -1] = 25000
    a[-1, :, :] = 15000
    nz, ny, nx = shape
    tf = _tf_dev(synth.default_tf(sigma_scale=0.3))
    cams = np.concatenate([synth.turntable_cameras(nx, ny, nz, n_views=6),
                           _grazing_cameras(nx, ny, nz)[::3]])
    v = to_dev_u16(a)
    lin = vr.vr_raycast(v, tf, cams, 48, 40, 0.5)
    if edge == 3:             # 4^3 bricks overlapping in x
        bv = vr.vr_brick_volume(v, overlap=True)
        br = _ovl_ref(a, pad_value=65535)[0]
    else:
        bv = vr.vr_brick_volume(v, edge=edge)
        e = edge
        nbz, nby, nbx = (nz + e - 1) // e, (ny + e - 1) // e, (nx + e - 1) // e
        pad = np.full((nbz * e, nby * e, nbx * e), 65535, dtype=np.uint16)
        pad[:nz, :ny, :nx] = a
        br = pad.reshape(nbz, e, nby, e, nbx, e).transpose(0, 2, 4, 1, 3, 5).reshape(-1)
        br = np.concatenate([br, np.full((nbx * nby + nbx + 1) * e ** 3, 65535, dtype=np.uint16)])
    assert br.size == bv.data.numel()
    bv.data.copy_(to_dev_u16(br))
    assert torch.equal(lin, vr.vr_raycast(bv, tf, cams, 48, 40, 0.5))
    assert lin[..., 3].max().item() > 0.1


def _grazing_cameras(nx, ny, nz):
    """Views whose rays run almost parallel to brick faces (tiny direction
    components), and exactly along an axis through brick boundaries."""
    c = np.array([nx, ny, nz], dtype=np.float64) / 2
    cams = []
    for tilt in (0.0, 1e-6, 3e-4, 2e-3):
        for axis in range(3):
            d = np.full(3, tilt)
            d[axis] = 1.0
            d /= np.linalg.norm(d)
            cam = np.zeros(11)
            cam[0:3] = c - 3.0 * max(nx, ny, nz) * d
            cam[3:6] = c
            cam[6:9] = (0.0, 0.0, 1.0) if axis != 2 else (0.0, 1.0, 0.0)
            cam[10] = 0.5 * max(nx, ny, nz)           # orthographic: rays on a grid through boundaries
            cams.append(cam)
            p = cam.copy()
            p[9], p[10] = 20.0, 0.0                   # and a narrow perspective view
            cams.append(p)
    return np.array(cams)


@pytest.mark.parametrize("shape", [(40, 36, 44), (33, 48, 29)])
def test_skip_exact_on_grazing_rays(shape):
    banner(f"grazing rays {shape}")
    a = _sparse_volume(shape, 9)
    nz, ny, nx = shape
    tf = _tf_dev(synth.default_tf(sigma_scale=3.0))
    cams = _grazing_cameras(nx, ny, nz)
    v = to_dev_u16(a)
    lin = vr.vr_raycast(v, tf, cams, 64, 64, 0.5)
    assert torch.equal(lin, vr.vr_raycast(vr.vr_brick_volume(v), tf, cams, 64, 64, 0.5))
    assert torch.equal(lin, vr.vr_raycast(vr.vr_brick_volume(v, pairs=True), tf, cams, 64, 64, 0.5))
    assert lin[..., 3].max().item() > 0.1


def test_skip_disabled_when_density_zero_is_not_empty(level1):
    banner("no skipping when tf[0] has extinction")
    tf = synth.default_tf()
    tf[0, 3] = 0.01                                   # density 0 now attenuates
    cams = synth.turntable_cameras(64, 64, 64, n_views=2)
    v = to_dev_u16(level1)
    lin = vr.vr_raycast(v, _tf_dev(tf), cams, 32, 32, 0.5)
    br = vr.vr_raycast(vr.vr_brick_volume(v), _tf_dev(tf), cams, 32, 32, 0.5)
    assert torch.equal(lin, br)
    ref, _ = R.render(level1, (1, 1, 1), tf.astype(np.float64), cams, 32, 32, 0.5)
    assert np.abs(br.cpu().numpy() - ref).max() <= TOL


def _zero_knots(tf):
    """Leading TF knots with zero extinction and finite colour."""
    ok = (tf[:, 3] == 0) & np.isfinite(tf[:, :3]).all(axis=1)
    return 256 if ok.all() else int(np.argmin(ok))


@pytest.mark.parametrize("shape", [(29, 23, 37), (64, 64, 64), (90, 70, 110)])
def test_tf_marked_occupancy_bit_identical(level1, shape):
    """Bricks marked only by voxels above the level the TF leaves at zero extinction:
    the occupancy is that of the volume with those voxels zeroed, and the frames and
    taken counts equal the linear march's bit for bit (4^3, 8^3 and pair bricks)."""
    banner(f"TF-marked occupancy {shape}")
    a = level1 if shape == (64, 64, 64) else _sparse_volume(shape, 11)
    nz, ny, nx = a.shape
    tf_h = synth.default_tf(sigma_scale=3.0)
    z = _zero_knots(tf_h)
    V = vr.tf_mark_level(tf_h)
    assert z >= 2 and V == 257 * (z - 1) - 1
    # every sample of taps <= V looks up knots below z - 1 (exact arithmetic)
    assert V * 255 / 65535 < z - 1
    tf = _tf_dev(tf_h)
    cams = np.concatenate([synth.turntable_cameras(nx, ny, nz, n_views=7),
                           synth.front_ortho_camera(nx, ny, nz)])
    v = to_dev_u16(a)
    c0 = torch.zeros(2, dtype=torch.int64, device=dev())
    lin = vr.vr_raycast(v, tf, cams, 45, 38, 0.5, samples=c0)
    below = np.where(a > V, a, 0).astype(np.uint16)
    fewer = []
    for kw in ({}, {"edge": 8}, {"pairs": True}):
        layout = vr.LAYOUT_BRICK8 if "edge" in kw else vr.LAYOUT_BRICK4_PAIRS if kw else vr.LAYOUT_BRICK4
        b0 = vr.vr_brick_volume(v, **kw)
        bm = vr.vr_brick_volume(v, mark_above=V, **kw)
        assert bm.mark_above == V and torch.equal(b0.data, bm.data)
        ref = vr.vr_brick_volume(to_dev_u16(below), **kw)
        assert torch.equal(_occ_parts_t(bm.occupancy, a.shape, layout), _occ_parts_t(ref.occupancy, a.shape, layout))
        c1 = torch.zeros(2, dtype=torch.int64, device=dev())
        c2 = torch.zeros(2, dtype=torch.int64, device=dev())
        f0 = vr.vr_raycast(b0, tf, cams, 45, 38, 0.5, samples=c1)
        fm = vr.vr_raycast(bm, tf, cams, 45, 38, 0.5, samples=c2)
        assert torch.equal(lin, f0) and torch.equal(lin, fm)
        if not kw:
            assert torch.equal(lin, vr.vr_raycast(bm, tf, cams, 45, 38, 0.5, staged=True))
        assert c2[0].item() == c1[0].item() == c0[0].item()
        assert c2[1].item() <= c1[1].item()
        fewer.append(c2[1].item() < c1[1].item())
    if shape != (64, 64, 64):
        assert all(fewer)                 # the blobs' faint tails no longer hold bricks open
    if shape == (29, 23, 37):
        _ref_occ = _brick_ref(below)[1]
        bm = vr.vr_brick_volume(v, mark_above=V)
        assert (_occ_parts(bm.occupancy, a.shape) == _ref_occ).all()


def _occ_parts_t(occ_t, shape, layout):
    nz, ny, nx = shape
    nb, _, nocc = vr.vr_brick_count_layout(layout, nx, ny, nz)
    return occ_t[:nocc - nb]


def test_tf_marked_occupancy_checked_against_the_tf():
    """Bricks marked for one TF, rendered with a TF that gives extinction to a knot
    their unmarked samples can reach: the ray caster marches every sample (frames
    equal to the linear march's, nothing passed over); a TF whose extinction starts
    just past that reach still passes them over."""
    banner("TF-marked occupancy under another TF")
    shape = (40, 36, 44)
    a = _sparse_volume(shape, 3)
    nz, ny, nx = shape
    tf_h = synth.default_tf(sigma_scale=3.0)
    z = _zero_knots(tf_h)
    V = vr.tf_mark_level(tf_h)
    cams = synth.turntable_cameras(nx, ny, nz, n_views=3)
    v = to_dev_u16(a)
    bm = vr.vr_brick_volume(v, mark_above=V)
    for knot, skips in ((z - 1, False), (z - 2, False), (0, False), (z, True)):
        bad = tf_h.copy()
        bad[knot, 3] = 0.05
        tf = _tf_dev(bad)
        c = torch.zeros(2, dtype=torch.int64, device=dev())
        lin = vr.vr_raycast(v, tf, cams, 40, 40, 0.5)
        got = vr.vr_raycast(bm, tf, cams, 40, 40, 0.5, samples=c)
        assert torch.equal(lin, got), knot
        assert (c[1].item() < c[0].item()) == skips, (knot, c)


@pytest.mark.parametrize("shape", [(64, 64, 64), (37, 60, 83), (70, 33, 81)])
def test_staged_march_bit_identical(level1, shape):
    """The depth-window march with LDS staging gives the gather march's frames, sample
    counts and grey-value counts bit for bit (perspective and orthographic views, a
    sparse volume with empty space, odd shapes, background)."""
    banner(f"staged march == gather march {shape}")
    a = level1 if shape == (64, 64, 64) else _sparse_volume(shape, 7)
    nz, ny, nx = a.shape
    tf = _tf_dev(synth.default_tf(sigma_scale=3.0))
    cams = np.concatenate([synth.turntable_cameras(nx, ny, nz, n_views=9),
                           synth.front_ortho_camera(nx, ny, nz)])
    bv = vr.vr_brick_volume(to_dev_u16(a))
    outs = []
    for staged in (False, True):
        cnt = torch.zeros(2, dtype=torch.int64, device=dev())
        vh = torch.zeros((len(cams), 256), dtype=torch.int32, device=dev())
        img = vr.vr_raycast(bv, tf, cams, 45, 38, 0.5, bg=BG, samples=cnt, view_hist=vh, staged=staged)
        outs.append((img, cnt, vh))
    assert torch.equal(outs[0][0], outs[1][0])
    assert torch.equal(outs[0][1], outs[1][1])
    assert torch.equal(outs[0][2], outs[1][2])


def test_staged_march_rejects_other_volumes(level1):
    v = to_dev_u16(level1)
    tf = _tf_dev(synth.default_tf())
    cam = synth.front_ortho_camera(64, 64, 64)
    with pytest.raises(vr.VrError):
        vr.vr_raycast(v, tf, cam, 8, 8, 0.5, staged=True)                 # linear layout
    with pytest.raises(vr.VrError):
        vr.vr_raycast(vr.vr_brick_volume(v, with_occupancy=False), tf, cam, 8, 8, 0.5, staged=True)
    f = torch.from_numpy(level1.astype(np.float32) / 65535.0).to(dev())
    with pytest.raises(vr.VrError):
        vr.vr_raycast(vr.vr_brick_volume(f), tf, cam, 8, 8, 0.5, staged=True)
