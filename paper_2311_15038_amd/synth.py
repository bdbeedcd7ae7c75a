"""Seeded synthetic micro-CT volumes.

The paper evaluates on five NOVA arthropod scans (Table II) that are not
public.  These generators stand in for them: a 16-bit volume of air around a
specimen made of nested ellipsoids and thin tubes, with per-class noise, and
both three-slice end slabs left as pure air (the histogram-filtering step of
Section III-D assumes the top slices hold only the surroundings).  Optionally
the specimen stands in a cylindrical container (a plastic wall about the z
axis over every slice, Section III-B), which the top slices then show as a
ring.

This module holds no step of the preview method itself: it only draws inputs.
Primitive geometry is drawn with NumPy's PCG64 from the seed, so it is the
same on every device; the per-voxel noise is drawn with a torch Generator on
the device the volume is built on (CPU and GPU noise streams differ).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import torch

# class id -> (mean grey value, noise sigma); ids index these tables.
AIR, OUTER, MIDDLE, INNER, TUBE, CONTAINER = 0, 1, 2, 3, 4, 5
CLASS_MU = (1000.0, 8000.0, 15000.0, 30000.0, 22000.0, 7000.0)
CLASS_SIGMA = (40.0, 300.0, 400.0, 500.0, 450.0, 300.0)

BASE = 128.0          # primitives are defined in a 128^3 base frame
END_SLAB = 3          # slices at each z end that stay pure air


@dataclass
class VolumeSpec:
    nx: int
    ny: int
    nz: int
    seed: int
    n_tubes: int = 20
    n_extra: int = 0              # extra random blobs/tubes (the 1024^3 scene)
    noise: str = "gauss"          # "gauss" or "poisson64"
    semi_axes: tuple = (50.0, 30.0, 12.0)
    aspect: tuple = (1.0, 0.8, 0.65)
    tube_radius: float = 2.0
    # cylindrical container: (centre x, centre y, inner radius, wall thickness)
    # in the base frame, over all slices; None = no container
    container: tuple | None = None

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)


SMALL = VolumeSpec(128, 128, 128, seed=2311)
FULL = VolumeSpec(1024, 1024, 1024, seed=2312, n_extra=477, noise="poisson64")
# the small and full scenes with a smaller specimen standing in a container
CONTAINER_RING = (64.6, 63.3, 60.0, 3.0)
SMALL_CONTAINED = VolumeSpec(128, 128, 128, seed=2313, semi_axes=(40.0, 24.0, 9.0),
                             container=CONTAINER_RING)
FULL_CONTAINED = VolumeSpec(1024, 1024, 1024, seed=2314, n_extra=477, noise="poisson64",
                            semi_axes=(40.0, 24.0, 9.0), container=CONTAINER_RING)


@dataclass
class _Prim:
    kind: str                     # "ell" or "tube"
    label: int
    a: np.ndarray                 # ellipsoid centre / tube end A (base frame)
    b: np.ndarray = field(default_factory=lambda: np.zeros(3))  # semi-axes / tube end B
    r: float = 0.0                # tube radius


def _primitives(spec: VolumeSpec):
    rng = np.random.Generator(np.random.PCG64(spec.seed))
    c = np.array([BASE / 2] * 3)
    asp = np.array(spec.aspect)
    prims = []
    for lab, r in zip((OUTER, MIDDLE, INNER), spec.semi_axes):
        prims.append(_Prim("ell", lab, c.copy(), r * asp))
    outer = spec.semi_axes[0] * asp
    lo, hi = c - outer, c + outer
    for _ in range(spec.n_tubes):
        p0, p1 = rng.uniform(lo, hi), rng.uniform(lo, hi)
        prims.append(_Prim("tube", TUBE, p0, p1, spec.tube_radius))
    for k in range(spec.n_extra):
        lab = int(rng.integers(OUTER, TUBE + 1))
        if k % 2 == 0:
            ctr = rng.uniform(lo, hi)
            ax = rng.uniform(1.0, 6.0, size=3)
            prims.append(_Prim("ell", lab, ctr, ax))
        else:
            p0, p1 = rng.uniform(lo, hi), rng.uniform(lo, hi)
            prims.append(_Prim("tube", lab, p0, p1, float(rng.uniform(0.25, 1.0))))
    return prims


def _index_range(lo_base, hi_base, scale, n):
    # voxel i has its centre at (i + 0.5) / scale in the base frame
    i0 = max(0, int(math.floor(lo_base * scale - 0.5)))
    i1 = min(n, int(math.ceil(hi_base * scale - 0.5)) + 1)
    return i0, i1


def _paint_container(lab: torch.Tensor, spec: VolumeSpec, sc):
    """The container wall: voxel centres whose base-frame distance from the
    axis lies in [inner radius, inner radius + thickness], in every slice."""
    cx, cy, r0, w = spec.container
    dev = lab.device
    xs = (torch.arange(spec.nx, device=dev, dtype=torch.float64) + 0.5) / float(sc[0]) - cx
    ys = (torch.arange(spec.ny, device=dev, dtype=torch.float64) + 0.5) / float(sc[1]) - cy
    d2 = xs[None, :] ** 2 + ys[:, None] ** 2
    ring = (d2 >= r0 * r0) & (d2 <= (r0 + w) ** 2)
    lab.masked_fill_(ring[None, :, :], CONTAINER)


def make_labels(spec: VolumeSpec, device="cpu") -> torch.Tensor:
    """Class id per voxel, int8 [nz][ny][nx]; later primitives paint over earlier ones."""
    dev = torch.device(device)
    lab = torch.zeros(spec.shape, dtype=torch.int8, device=dev)
    sc = np.array([spec.nx, spec.ny, spec.nz], dtype=np.float64) / BASE
    n = (spec.nx, spec.ny, spec.nz)
    if spec.container is not None:
        _paint_container(lab, spec, sc)
    zlo, zhi = END_SLAB, spec.nz - END_SLAB
    if zhi <= zlo:
        return lab
    for p in _primitives(spec):
        if p.kind == "ell":
            blo, bhi = p.a - p.b, p.a + p.b
        else:
            blo = np.minimum(p.a, p.b) - p.r
            bhi = np.maximum(p.a, p.b) + p.r
        rng3 = [_index_range(blo[k], bhi[k], sc[k], n[k]) for k in range(3)]
        (x0, x1), (y0, y1), (z0, z1) = rng3
        z0, z1 = max(z0, zlo), min(z1, zhi)
        if x1 <= x0 or y1 <= y0 or z1 <= z0:
            continue
        xs = (torch.arange(x0, x1, device=dev, dtype=torch.float32) + 0.5) / float(sc[0])
        ys = (torch.arange(y0, y1, device=dev, dtype=torch.float32) + 0.5) / float(sc[1])
        zs = (torch.arange(z0, z1, device=dev, dtype=torch.float32) + 0.5) / float(sc[2])
        X, Y, Z = xs[None, None, :], ys[None, :, None], zs[:, None, None]
        if p.kind == "ell":
            m = (((X - float(p.a[0])) / float(p.b[0])) ** 2
                 + ((Y - float(p.a[1])) / float(p.b[1])) ** 2
                 + ((Z - float(p.a[2])) / float(p.b[2])) ** 2) <= 1.0
        else:
            d = p.b - p.a
            dd = float(np.dot(d, d))
            px, py, pz = X - float(p.a[0]), Y - float(p.a[1]), Z - float(p.a[2])
            t = (px * float(d[0]) + py * float(d[1]) + pz * float(d[2])) / max(dd, 1e-12)
            t = t.clamp(0.0, 1.0)
            ex = px - t * float(d[0])
            ey = py - t * float(d[1])
            ez = pz - t * float(d[2])
            m = (ex * ex + ey * ey + ez * ez) <= p.r * p.r
        sub = lab[z0:z1, y0:y1, x0:x1]
        sub.masked_fill_(m, p.label)
    return lab


def make_volume(spec: VolumeSpec, device="cpu") -> torch.Tensor:
    """uint16 volume [nz][ny][nx], x fastest, on `device`."""
    dev = torch.device(device)
    lab = make_labels(spec, dev).long()
    mu = torch.tensor(CLASS_MU, dtype=torch.float32, device=dev)[lab]
    sg = torch.tensor(CLASS_SIGMA, dtype=torch.float32, device=dev)[lab]
    del lab
    g = torch.Generator(device=dev)
    g.manual_seed(spec.seed)
    if spec.noise == "gauss":
        v = torch.randn(spec.shape, generator=g, device=dev, dtype=torch.float32)
        v.mul_(sg).add_(mu)
    elif spec.noise == "poisson64":
        v = torch.poisson(mu / 64.0, generator=g).mul_(64.0)
        nrm = torch.randn(spec.shape, generator=g, device=dev, dtype=torch.float32)
        v.add_(nrm.mul_(sg))
        del nrm
    else:
        raise ValueError(f"unknown noise model {spec.noise!r}")
    del mu, sg
    v = torch.round(v).clamp_(0.0, 65535.0)
    return v.to(torch.int32).to(torch.uint16)


def scaled_spec(nx, ny, nz, seed, noise="gauss") -> VolumeSpec:
    """The small scene stretched per axis to nx x ny x nz (uneven batch volumes)."""
    return VolumeSpec(nx, ny, nz, seed=seed, noise=noise)


def batch_specs(count=64, seed=3000, lo=64, hi=512):
    """Uneven anisotropic volumes, each axis uniform on [lo, hi]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(count):
        nx, ny, nz = (int(v) for v in rng.integers(lo, hi + 1, size=3))
        out.append(scaled_spec(nx, ny, nz, seed + i))
    return out


def to_numpy_u16(t: torch.Tensor) -> np.ndarray:
    return t.cpu().view(torch.int16).numpy().view(np.uint16)


def from_numpy_u16(a: np.ndarray, device="cpu") -> torch.Tensor:
    a = np.ascontiguousarray(a, dtype=np.uint16)
    return torch.from_numpy(a.view(np.int16)).view(torch.uint16).to(device)


# ------------------------------------------------------------- views and TF
# A camera is a row of 11 numbers: eye[3], target[3], up[3], vertical field of
# view in degrees (> 0: perspective) and the orthographic half height (used
# when the field of view is 0).  World units: voxel index times spacing.

def _box(nx, ny, nz, spacing):
    ext = np.array([nx, ny, nz], dtype=np.float64) * np.asarray(spacing, dtype=np.float64)
    return ext / 2.0, 0.5 * float(np.linalg.norm(ext))


def turntable_cameras(nx, ny, nz, spacing=(1.0, 1.0, 1.0), n_views=36, fov_deg=60.0):
    """Views k = 0..n_views-1 on a circle about +z through the box centre
    (the Z-axis rotation of the server-side snapshots), at twice the box's
    half diagonal from the centre."""
    c, rho = _box(nx, ny, nz, spacing)
    cams = np.zeros((n_views, 11), dtype=np.float64)
    for k in range(n_views):
        th = 2.0 * math.pi * k / n_views
        cams[k, 0:3] = c + 2.0 * rho * np.array([math.cos(th), math.sin(th), 0.0])
        cams[k, 3:6] = c
        cams[k, 6:9] = (0.0, 0.0, 1.0)
        cams[k, 9] = fov_deg
    return cams


def front_ortho_camera(nx, ny, nz, spacing=(1.0, 1.0, 1.0)):
    """One orthographic view along +y whose square view just covers the box."""
    c, rho = _box(nx, ny, nz, spacing)
    cam = np.zeros((1, 11), dtype=np.float64)
    cam[0, 0:3] = c - 2.0 * rho * np.array([0.0, 1.0, 0.0])
    cam[0, 3:6] = c
    cam[0, 6:9] = (0.0, 0.0, 1.0)
    cam[0, 10] = 0.5 * max(nx * spacing[0], nz * spacing[2])
    return cam


# (s, r, g, b, sigma per world unit) anchors; s = grey / 65535.  sigma is zero
# below s = 0.06 so removed and air voxels are empty, and rises through the
# class means (outer shell translucent, dense core opaque).
TF_ANCHORS = (
    (0.000, 0.00, 0.00, 0.00, 0.00),
    (0.060, 0.00, 0.00, 0.00, 0.00),
    (0.122, 0.90, 0.60, 0.30, 0.02),
    (0.229, 0.30, 0.80, 0.40, 0.08),
    (0.336, 0.30, 0.50, 0.90, 0.15),
    (0.458, 1.00, 1.00, 0.90, 0.50),
    (1.000, 1.00, 1.00, 1.00, 0.50),
)


def default_tf(sigma_scale=1.0) -> np.ndarray:
    """256 x 4 float32 table (r, g, b, sigma) sampled from TF_ANCHORS at s = k/255."""
    a = np.array(TF_ANCHORS, dtype=np.float64)
    s = np.arange(256) / 255.0
    tf = np.stack([np.interp(s, a[:, 0], a[:, c]) for c in range(1, 5)], axis=1)
    tf[:, 3] *= sigma_scale
    return tf.astype(np.float32)


def random_tf(seed, sigma_max=0.5) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    tf = rng.uniform(0.0, 1.0, size=(256, 4))
    tf[:, 3] *= sigma_max
    return tf.astype(np.float32)
