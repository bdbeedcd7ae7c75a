"""Python side of the FP64 ray-casting oracle (TEST INFRASTRUCTURE ONLY).

Loads oracle/liboracle_render.so (plain C, gcc, OpenMP over rays), building it
with gcc when it is missing.  Cameras are rows of 11 numbers: eye[3],
target[3], up[3], vertical field of view in degrees (> 0 perspective) and the
orthographic half height (used when the field of view is 0).

Sample counts come with bounds: a renderer that takes the step count
ceil(L/step) and the early-termination test T < ert_eps in lower precision
may decide either one differently, by one sample, on rays where the decision
lies within COUNT_TOL (relative) of its boundary.  [lo, hi] is the count with
both decisions moved to the edges of that margin (see render.c).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "render.c")
_SO = os.path.join(_HERE, "liboracle_render.so")
_lib = None

U16, F32, F64 = 0, 1, 2
COUNT_TOL = 2.0 ** -10


class _Vol(C.Structure):
    _fields_ = [("data", C.c_void_p), ("dtype", C.c_int), ("nx", C.c_long),
                ("ny", C.c_long), ("nz", C.c_long), ("spacing", C.c_double * 3)]


class _Cam(C.Structure):
    _fields_ = [("eye", C.c_double * 3), ("target", C.c_double * 3), ("up", C.c_double * 3),
                ("fov_y_deg", C.c_double), ("ortho_half_h", C.c_double)]


def build():
    cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
           "-o", _SO + ".tmp", _SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(_SO + ".tmp", _SO)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = C.CDLL(_SO)
        P = C.POINTER
        L.or_render.argtypes = [P(_Vol), P(C.c_double), P(_Cam), C.c_int, C.c_int, C.c_int,
                                C.c_double, C.c_double, P(C.c_double), P(C.c_double),
                                P(C.c_longlong), C.c_double, P(C.c_longlong)]
        L.or_render_pixels.argtypes = [P(_Vol), P(C.c_double), P(_Cam), C.c_int, C.c_int,
                                       C.c_double, C.c_double, P(C.c_double), C.c_long,
                                       P(C.c_int32), P(C.c_double), P(C.c_longlong),
                                       C.c_double, P(C.c_longlong)]
        L.or_density_many.argtypes = [P(_Vol), C.c_long, P(C.c_double), P(C.c_double)]
        L.or_threads.restype = C.c_int
        _lib = L
    return _lib


def threads() -> int:
    return int(lib().or_threads())


def _ptr(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def _volume(vol, spacing):
    vol = np.ascontiguousarray(vol)
    dt = {np.dtype(np.uint16): U16, np.dtype(np.float32): F32, np.dtype(np.float64): F64}[vol.dtype]
    nz, ny, nx = vol.shape
    v = _Vol(vol.ctypes.data, dt, nx, ny, nz, (C.c_double * 3)(*[float(s) for s in spacing]))
    return v, vol


def _cams(cams):
    cams = np.asarray(cams, dtype=np.float64).reshape(-1, 11)
    arr = (_Cam * len(cams))()
    for k, c in enumerate(cams):
        arr[k].eye[:] = list(c[0:3])
        arr[k].target[:] = list(c[3:6])
        arr[k].up[:] = list(c[6:9])
        arr[k].fov_y_deg = float(c[9])
        arr[k].ortho_half_h = float(c[10])
    return arr, len(cams)


def render(vol, spacing, tf, cams, W, H, step, ert_eps=2.0 ** -14, bg=(0.0, 0.0, 0.0, 0.0),
           bounds=False):
    """FP64 render of every pixel of every view -> (rgba [V][H][W][4], samples [V]),
    and with bounds=True also the count bounds [V][2] = (lo, hi) under COUNT_TOL."""
    v, keep = _volume(vol, spacing)
    tf = np.ascontiguousarray(tf, dtype=np.float64).reshape(256, 4)
    ca, nv = _cams(cams)
    bga = np.asarray(bg, dtype=np.float64)
    out = np.zeros((nv, H, W, 4), dtype=np.float64)
    samples = np.zeros(nv, dtype=np.int64)
    lohi = np.zeros((nv, 2), dtype=np.int64)
    lib().or_render(C.byref(v), _ptr(tf, C.c_double), ca, nv, W, H, float(step), float(ert_eps),
                    _ptr(bga, C.c_double), _ptr(out, C.c_double), _ptr(samples, C.c_longlong),
                    COUNT_TOL, _ptr(lohi, C.c_longlong))
    del keep
    return (out, samples, lohi) if bounds else (out, samples)


def render_pixels(vol, spacing, tf, cams, W, H, step, pix, ert_eps=2.0 ** -14,
                  bg=(0.0, 0.0, 0.0, 0.0), per_pixel=False):
    """FP64 render of selected pixels pix[k] = (view, j, i) -> (rgba [K][4], samples),
    and with per_pixel=True also [K][3]: each pixel's count and its (lo, hi)."""
    v, keep = _volume(vol, spacing)
    tf = np.ascontiguousarray(tf, dtype=np.float64).reshape(256, 4)
    ca, _ = _cams(cams)
    bga = np.asarray(bg, dtype=np.float64)
    pix = np.ascontiguousarray(pix, dtype=np.int32).reshape(-1, 3)
    out = np.zeros((len(pix), 4), dtype=np.float64)
    cnt = np.zeros(1, dtype=np.int64)
    counts = np.zeros((len(pix), 3), dtype=np.int64)
    lib().or_render_pixels(C.byref(v), _ptr(tf, C.c_double), ca, W, H, float(step),
                           float(ert_eps), _ptr(bga, C.c_double), len(pix), _ptr(pix, C.c_int32),
                           _ptr(out, C.c_double), _ptr(cnt, C.c_longlong), COUNT_TOL,
                           _ptr(counts, C.c_longlong))
    del keep
    return (out, int(cnt[0]), counts) if per_pixel else (out, int(cnt[0]))


def density_at(vol, spacing, pts):
    """The oracle's trilinear density at world points pts[k] = (x, y, z)."""
    v, keep = _volume(vol, spacing)
    pts = np.ascontiguousarray(pts, dtype=np.float64).reshape(-1, 3)
    out = np.zeros(len(pts), dtype=np.float64)
    lib().or_density_many(C.byref(v), len(pts), _ptr(pts, C.c_double), _ptr(out, C.c_double))
    del keep
    return out
