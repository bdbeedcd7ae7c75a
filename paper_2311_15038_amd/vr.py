"""ctypes binding of libvr.so: the C ABI declared in include/vr.h, same names.

Argument marshalling only: tensors are passed as device pointers, the stream
is torch's current HIP stream unless one is given, and every step of the path
runs in the library's HIP kernels.  If libvr.so is missing, or a call is made
without a GPU, the binding raises; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libvr.so")

NBINS = 65536
KEEP_WORDS = 2048
CIRCLE_INTS = 8
CONTAINER_SCRATCH_BYTES = 32 << 20
HOLLOW_MAX_THICKNESS = 8
MAX_LEVELS = 8
MAX_VIEWS_PER_LAUNCH = 48
BRICK_DIST_CAP = 8
RULE_VALLEY, RULE_OTSU, RULE_ITS, RULE_NONE = 0, 1, 2, 3
U16_NORM, F32 = 0, 1
LAYOUT_LINEAR, LAYOUT_BRICK4, LAYOUT_BRICK4_PAIRS, LAYOUT_BRICK8, LAYOUT_BRICK4_OVERLAP = 0, 1, 2, 3, 4
ERRORS = {-1: "VR_ERR_NULL", -2: "VR_ERR_DIMS", -3: "VR_ERR_RANGE", -4: "VR_ERR_DTYPE",
          -5: "VR_ERR_HIP", -6: "VR_ERR_UNSUPPORTED", -7: "VR_ERR_WORKSPACE"}


class VrError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class vr_volume(C.Structure):
    _fields_ = [("data", C.c_void_p), ("dtype", C.c_int32), ("layout", C.c_int32),
                ("nx", C.c_int64), ("ny", C.c_int64), ("nz", C.c_int64),
                ("spacing", C.c_double * 3), ("occupancy", C.c_void_p), ("occupancy_above", C.c_int32)]


class vr_camera(C.Structure):
    _fields_ = [("eye", C.c_double * 3), ("target", C.c_double * 3), ("up", C.c_double * 3),
                ("fov_y_deg", C.c_double), ("ortho_half_h", C.c_double)]


class vr_atlas_spec(C.Structure):
    _fields_ = [("level", C.c_int32), ("tiles_x", C.c_int32), ("tiles_y", C.c_int32),
                ("out_bits", C.c_int32), ("data", C.c_void_p)]


class vr_batch_item(C.Structure):
    _fields_ = [("d_vol", C.c_void_p), ("nx", C.c_int64), ("ny", C.c_int64), ("nz", C.c_int64),
                ("spacing", C.c_double * 3), ("n_views", C.c_int32), ("h_cams", C.c_void_p),
                ("d_frames", C.c_void_p)]


class vr_batch_config(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("step", C.c_float),
                ("ert_eps", C.c_float), ("bg", C.c_float * 4), ("rule", C.c_int32),
                ("rule_param", C.c_int32), ("top_slices", C.c_int32), ("wave_w", C.c_int32),
                ("wave_h", C.c_int32), ("waves_x", C.c_int32), ("hist_task_voxels", C.c_int64),
                ("down_tiles_per_task", C.c_int32), ("slabs_per_task", C.c_int32),
                ("render_tiles_per_task", C.c_int32), ("brick_edge", C.c_int32)]


class vr_render_opts(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("step", C.c_float),
                ("ert_eps", C.c_float), ("bg", C.c_float * 4), ("view_hist", C.c_void_p),
                ("flags", C.c_uint32)]


RENDER_STAGED = 1


_lib = None


def lib():
    """The loaded library; raises if libvr.so has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2311_15038_amd.build` (no CPU fallback exists)")
        L = C.CDLL(LIB_PATH)
        vp, i64, i32 = C.c_void_p, C.c_int64, C.c_int
        L.vr_histogram.argtypes = [vp, i64, i64, i64, i64, i64, vp, vp]
        L.vr_select_threshold.argtypes = [vp, vp, i32, i32, vp, vp, vp]
        L.vr_threshold_downsample.argtypes = [vp, i64, i64, i64, vp, i32, C.POINTER(vp), C.POINTER(vp),
                                              C.POINTER(vr_atlas_spec), vp]
        L.vr_histogram_with_top.argtypes = [vp, i64, i64, i64, i64, vp, vp, vp]
        L.vr_container_workspace_size.argtypes = [i64, i64, i32, C.POINTER(C.c_int64)]
        L.vr_find_container.argtypes = [vp, i64, i64, i32, i32, i32, i32, vp, i64, vp, vp]
        L.vr_find_container_noalloc.argtypes = [vp, i64, i64, i32, i32, i32, i32, vp, vp]
        L.vr_remove_container.argtypes = [vp, i64, i64, i64, vp, vp]
        L.vr_hollow.argtypes = [vp, i64, i64, i64, i32, vp, vp, vp]
        L.vr_histogram_in_disc.argtypes = [vp, i64, i64, i64, i64, vp, vp, vp, vp]
        L.vr_threshold_downsample_in_disc.argtypes = [vp, i64, i64, i64, vp, vp, i32, C.POINTER(vp),
                                                      C.POINTER(vp), C.POINTER(vr_atlas_spec), vp]
        L.vr_pack_slicemap.argtypes = [vp, i64, i64, i64, i32, i32, i32, vp, vp]
        L.vr_raycast.argtypes = [C.POINTER(vr_volume), vp, C.POINTER(vr_camera), i32,
                                 C.POINTER(vr_render_opts), vp, vp, vp]
        L.vr_raycast_backward.argtypes = [C.POINTER(vr_volume), vp, C.POINTER(vr_camera), i32,
                                          C.POINTER(vr_render_opts), vp, vp, vp, vp, vp]
        L.vr_brick_volume.argtypes = [vp, i32, i32, i64, i64, i64, vp, vp, i32, vp]
        L.vr_unbrick_volume.argtypes = [vp, i32, i64, i64, i64, vp, vp]
        L.vr_frame_entropy.argtypes = [vp, i32, i32, i32, vp, vp, vp, vp]
        L.vr_entropy_from_counts.argtypes = [vp, i32, i64, vp, vp, vp]
        L.vr_brick_count.argtypes = [i64, i64, i64, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
        L.vr_brick_count_layout.argtypes = [i32, i64, i64, i64, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                            C.POINTER(C.c_int64)]
        PB = C.POINTER(vr_batch_item)
        PC = C.POINTER(vr_batch_config)
        L.vr_batch_workspace_size.argtypes = [PB, i32, PC, C.POINTER(C.c_int64)]
        L.vr_batch_plan_create.argtypes = [PB, i32, PC, vp, vp, i64, C.POINTER(vp)]
        L.vr_batch_launch.argtypes = [vp, vp]
        L.vr_batch_capture.argtypes = [vp, vp]
        L.vr_batch_status.argtypes = [vp, C.POINTER(C.c_uint32), C.POINTER(C.c_uint64)]
        L.vr_batch_item_outputs.argtypes = [vp, i32, C.POINTER(vp), C.POINTER(vp), C.POINTER(C.c_int64)]
        L.vr_batch_plan_destroy.argtypes = [vp]
        L.vr_last_error.restype = C.c_char_p
        L.vr_version.restype = C.c_char_p
        for name in ("vr_histogram", "vr_select_threshold", "vr_threshold_downsample",
                     "vr_pack_slicemap", "vr_raycast", "vr_raycast_backward", "vr_brick_volume",
                     "vr_unbrick_volume", "vr_frame_entropy", "vr_entropy_from_counts", "vr_container_workspace_size",
                     "vr_find_container", "vr_find_container_noalloc", "vr_remove_container", "vr_histogram_in_disc",
                     "vr_threshold_downsample_in_disc", "vr_hollow",
                     "vr_brick_count", "vr_brick_count_layout", "vr_histogram_with_top", "vr_batch_workspace_size",
                     "vr_batch_plan_create", "vr_batch_launch", "vr_batch_capture", "vr_batch_status",
                     "vr_batch_item_outputs", "vr_batch_plan_destroy"):
            getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _check(rc):
    if rc != 0:
        raise VrError(rc, lib().vr_last_error().decode())


def _stream(stream):
    if stream is None:
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, torch.cuda.Stream):
        return C.c_void_p(stream.cuda_stream)
    return C.c_void_p(int(stream))


def _dev(t: torch.Tensor, name: str, dtype=None, numel=None):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype not in (dtype if isinstance(dtype, tuple) else (dtype,)):
        raise TypeError(f"{name} has dtype {t.dtype}, expected {dtype}")
    if numel is not None and t.numel() < numel:
        raise ValueError(f"{name} holds {t.numel()} elements, needs {numel}")
    return C.c_void_p(t.data_ptr())


_U16 = (torch.uint16, torch.int16)


def version() -> str:
    return lib().vr_version().decode()


# ------------------------------------------------------------------ reduction
def vr_histogram(vol, z0=0, nz_range=None, out=None, stream=None):
    """uint16 volume [nz][ny][nx] -> 65536 counters (int64 tensor holding the uint64 counts)."""
    nz, ny, nx = vol.shape
    if nz_range is None:
        nz_range = nz - z0
    if out is None:
        out = torch.empty(NBINS, dtype=torch.int64, device=vol.device)
    _check(lib().vr_histogram(_dev(vol, "vol", _U16), nx, ny, nz, z0, nz_range,
                              _dev(out, "out", torch.int64, NBINS), _stream(stream)))
    return out


def vr_histogram_with_top(vol, top_slices=3, hist=None, hist_top=None, stream=None):
    """Histograms of the whole volume and of its first top_slices slices, one launch."""
    nz, ny, nx = vol.shape
    if hist is None:
        hist = torch.empty(NBINS, dtype=torch.int64, device=vol.device)
    if hist_top is None:
        hist_top = torch.empty(NBINS, dtype=torch.int64, device=vol.device)
    _check(lib().vr_histogram_with_top(_dev(vol, "vol", _U16), nx, ny, nz, int(top_slices),
                                       _dev(hist, "hist", torch.int64, NBINS),
                                       _dev(hist_top, "hist_top", torch.int64, NBINS),
                                       _stream(stream)))
    return hist, hist_top


def vr_select_threshold(hist, hist_top=None, rule=RULE_VALLEY, param=32, result=None, keep_bits=None,
                        stream=None):
    """-> (result int32[4] = T, aux, b*, 0; keep_bits int32[2048] holding the uint32 mask)."""
    dev = hist.device
    if result is None:
        result = torch.empty(4, dtype=torch.int32, device=dev)
    if keep_bits is None:
        keep_bits = torch.empty(KEEP_WORDS, dtype=torch.int32, device=dev)
    top = None if hist_top is None else _dev(hist_top, "hist_top", torch.int64, NBINS)
    _check(lib().vr_select_threshold(_dev(hist, "hist", torch.int64, NBINS), top, int(rule),
                                     int(param), _dev(result, "result", torch.int32, 4),
                                     _dev(keep_bits, "keep_bits", torch.int32, KEEP_WORDS),
                                     _stream(stream)))
    return result, keep_bits


# ---------------------------------------------------------- container removal
def vr_container_workspace_size(nx, ny, r_max):
    b = C.c_int64(0)
    _check(lib().vr_container_workspace_size(int(nx), int(ny), int(r_max), C.byref(b)))
    return int(b.value)


def container_radii(nx, ny):
    """Default radius range of the container search: [min side / 8, min side / 2]."""
    m = min(nx, ny)
    return max(1, m // 8), max(1, m // 2)


def vr_find_container(slice2d, r_min=None, r_max=None, edge_shift=4, margin=2, work=None, circle=None,
                      stream=None):
    """Circle record (int32[8] on the device) of the container in a u16 slice [ny][nx]."""
    ny, nx = slice2d.shape
    lo, hi = container_radii(nx, ny)
    r_min = lo if r_min is None else r_min
    r_max = hi if r_max is None else r_max
    need = vr_container_workspace_size(nx, ny, r_max)
    if work is None:
        work = torch.empty(need, dtype=torch.uint8, device=slice2d.device)
    if circle is None:
        circle = torch.empty(CIRCLE_INTS, dtype=torch.int32, device=slice2d.device)
    _check(lib().vr_find_container(_dev(slice2d, "slice", _U16), nx, ny, int(r_min), int(r_max),
                                   int(edge_shift), int(margin), _dev(work, "work", torch.uint8, need),
                                   work.numel(), _dev(circle, "circle", torch.int32, CIRCLE_INTS),
                                   _stream(stream)))
    return circle


def vr_find_container_noalloc(slice2d, r_min=None, r_max=None, edge_shift=4, margin=2, circle=None,
                              stream=None):
    """vr_find_container with the library's fixed device scratch as its workspace
    (the call allocates nothing; pass `circle` to allocate nothing here either)."""
    ny, nx = slice2d.shape
    lo, hi = container_radii(nx, ny)
    r_min = lo if r_min is None else r_min
    r_max = hi if r_max is None else r_max
    if circle is None:
        circle = torch.empty(CIRCLE_INTS, dtype=torch.int32, device=slice2d.device)
    _check(lib().vr_find_container_noalloc(_dev(slice2d, "slice", _U16), nx, ny, int(r_min), int(r_max),
                                           int(edge_shift), int(margin),
                                           _dev(circle, "circle", torch.int32, CIRCLE_INTS), _stream(stream)))
    return circle


def vr_remove_container(vol, circle, stream=None):
    """Zero every voxel outside the kept disc, in place; returns vol."""
    nz, ny, nx = vol.shape
    _check(lib().vr_remove_container(_dev(vol, "vol", _U16), nx, ny, nz,
                                     _dev(circle, "circle", torch.int32, CIRCLE_INTS), _stream(stream)))
    return vol


def vr_hollow(vol, thickness, out=None, kept=None, stream=None):
    """Hollow data preview: the non-zero voxels within city-block distance
    `thickness` of a zero voxel or of the volume's outside keep their value,
    every other voxel is 0.  out: a new tensor unless given (must not overlap
    vol); kept: None or an int64 tensor of one element, overwritten with the
    number of kept voxels.  Returns out."""
    nz, ny, nx = vol.shape
    if out is None:
        out = torch.empty_like(vol)
    kp = None if kept is None else _dev(kept, "kept", torch.int64, 1)
    _check(lib().vr_hollow(_dev(vol, "vol", _U16), nx, ny, nz, int(thickness),
                           _dev(out, "out", _U16, nx * ny * nz), kp, _stream(stream)))
    return out


def vr_histogram_in_disc(vol, circle, top_slices=3, hist=None, hist_top=None, stream=None):
    """Histograms of the voxels inside the kept disc: the whole volume and its
    first top_slices slices (top_slices 0: no top histogram, returns None)."""
    nz, ny, nx = vol.shape
    if hist is None:
        hist = torch.empty(NBINS, dtype=torch.int64, device=vol.device)
    if hist_top is None and top_slices:
        hist_top = torch.empty(NBINS, dtype=torch.int64, device=vol.device)
    top = _dev(hist_top, "hist_top", torch.int64, NBINS) if top_slices else None
    _check(lib().vr_histogram_in_disc(_dev(vol, "vol", _U16), nx, ny, nz, int(top_slices),
                                      _dev(circle, "circle", torch.int32, CIRCLE_INTS),
                                      _dev(hist, "hist", torch.int64, NBINS), top, _stream(stream)))
    return hist, (hist_top if top_slices else None)


def level_shape(shape, k):
    d = 1 << k
    return tuple(-(-n // d) for n in shape)


def vr_threshold_downsample(vol, keep_bits, n_levels, levels=None, atlas=None, stream=None, circle=None,
                            sums=None):
    """Filtered pyramid levels 1..n_levels (list of uint16 tensors), or
    (levels, sums) when sums is given.

    atlas: None or (level, tiles_x, tiles_y, out_bits, tensor): the slicemap
    atlas of that level, written in the same pass.
    circle: None, or a container circle record (vr_find_container): voxels
    outside its kept disc count as removed (vr_threshold_downsample_in_disc).
    sums: None, True (one new int64 tensor of exact level sums per level), or a
    list of n_levels tensors (or None entries).  With more than four levels
    the level-4 sums are needed by the call: a buffer for them is made here
    when the caller does not ask for it.
    """
    nz, ny, nx = vol.shape
    if levels is None:
        levels = [torch.empty(level_shape((nz, ny, nx), k), dtype=torch.uint16, device=vol.device)
                  for k in range(1, n_levels + 1)]
    if len(levels) < n_levels:
        raise ValueError("need one output tensor per level")
    ptrs = (C.c_void_p * max(1, n_levels))()
    for k in range(n_levels):
        want = level_shape((nz, ny, nx), k + 1)
        if tuple(levels[k].shape) != want:
            raise ValueError(f"level {k + 1} has shape {tuple(levels[k].shape)}, expected {want}")
        ptrs[k] = _dev(levels[k], f"levels[{k}]", _U16).value
    kb = None if keep_bits is None else _dev(keep_bits, "keep_bits", torch.int32, KEEP_WORDS)
    want_sums = sums is not None
    if sums is True:
        sums = [torch.empty(level_shape((nz, ny, nx), k), dtype=torch.int64, device=vol.device)
                for k in range(1, n_levels + 1)]
    elif sums is None:
        sums = [None] * max(n_levels, 0)
    if len(sums) < n_levels:
        raise ValueError("need one sums entry per level")
    if n_levels > 4 and sums[3] is None:
        sums = list(sums)
        sums[3] = torch.empty(level_shape((nz, ny, nx), 4), dtype=torch.int64, device=vol.device)
    sptrs = None
    if any(t is not None for t in sums[:n_levels]):
        sptrs = (C.c_void_p * max(1, n_levels))()
        for k in range(n_levels):
            if sums[k] is not None:
                if tuple(sums[k].shape) != level_shape((nz, ny, nx), k + 1):
                    raise ValueError(f"sums {k + 1} has shape {tuple(sums[k].shape)}")
                sptrs[k] = _dev(sums[k], f"sums[{k}]", torch.int64).value
    spec = None
    if atlas is not None:
        lvl, tx, ty, bits, t = atlas
        lz, ly, lx = level_shape((nz, ny, nx), lvl)
        dt = (torch.uint16, torch.int16) if bits == 16 else torch.uint8
        spec = C.byref(vr_atlas_spec(int(lvl), int(tx), int(ty), int(bits),
                                     _dev(t, "atlas", dt, tx * ty * lx * ly).value))
    if circle is None:
        _check(lib().vr_threshold_downsample(_dev(vol, "vol", _U16), nx, ny, nz, kb, int(n_levels),
                                             ptrs, sptrs, spec, _stream(stream)))
    else:
        _check(lib().vr_threshold_downsample_in_disc(
            _dev(vol, "vol", _U16), nx, ny, nz, kb, _dev(circle, "circle", torch.int32, CIRCLE_INTS),
            int(n_levels), ptrs, sptrs, spec, _stream(stream)))
    return (levels, sums[:n_levels]) if want_sums else levels


def vr_pack_slicemap(level, tiles_x, tiles_y, out_bits=16, out=None, stream=None):
    nz, ny, nx = level.shape
    dt = torch.uint16 if out_bits == 16 else torch.uint8
    if out is None:
        out = torch.empty((tiles_y * ny, tiles_x * nx), dtype=dt, device=level.device)
    _check(lib().vr_pack_slicemap(_dev(level, "level", _U16), nx, ny, nz, int(tiles_x),
                                  int(tiles_y), int(out_bits),
                                  _dev(out, "out", (dt, torch.int16) if out_bits == 16 else dt,
                                       tiles_x * tiles_y * nx * ny),
                                  _stream(stream)))
    return out


# ------------------------------------------------------------------ rendering
def vr_brick_count_layout(layout, nx, ny, nz):
    """-> (bricks, elements of the bricked volume, bytes of the occupancy grids) of a brick layout."""
    n, e, o = C.c_int64(0), C.c_int64(0), C.c_int64(0)
    _check(lib().vr_brick_count_layout(int(layout), nx, ny, nz, C.byref(n), C.byref(e), C.byref(o)))
    return int(n.value), int(e.value), int(o.value)


def vr_brick_count(nx, ny, nz):
    """-> (number of 4^3 bricks, bytes of the occupancy grids)."""
    n, o = C.c_int64(0), C.c_int64(0)
    _check(lib().vr_brick_count(nx, ny, nz, C.byref(n), C.byref(o)))
    return int(n.value), int(o.value)


def tf_mark_level(tf) -> int:
    """A brick-marking level V (u16 units) for this TF under which samples of
    unmarked bricks (all eight taps at most V) leave its render unchanged: with
    the first z knots of zero extinction and finite colour, 257 (z - 1) - 1
    (z >= 2; such a sample's TF coordinate stays below z - 1), else 0.
    tf: [256][4] (r, g, b, sigma), host array or tensor."""
    a = np.asarray(tf.detach().cpu() if isinstance(tf, torch.Tensor) else tf, dtype=np.float64).reshape(256, 4)
    ok = (a[:, 3] == 0.0) & np.isfinite(a[:, :3]).all(axis=1)
    z = 256 if ok.all() else int(np.argmin(ok))
    return 257 * (z - 1) - 1 if z >= 2 else 0


class BrickedVolume:
    """A volume in a brick render layout (4^3 bricks, 4^3 bricks of x-tap pairs,
    or 8^3 bricks), with its occupancy grid (or None) and the level its marks
    are above (mark_above)."""

    def __init__(self, data, shape, occupancy=None, layout=None, mark_above=0):
        self.data, self.shape, self.occupancy = data, tuple(shape), occupancy
        self.layout = LAYOUT_BRICK4 if layout is None else layout
        self.mark_above = int(mark_above)
        self.dtype = data.dtype
        self.device = data.device


def vr_brick_volume(src, out=None, with_occupancy=True, stream=None, pairs=False, edge=4,
                    mark_above=0, overlap=False) -> BrickedVolume:
    """Copy a [nz][ny][nx] u16 or f32 volume into the brick layout (+ occupancy):
    bricks of `edge` (4 or 8) voxels; with pairs, the 4^3 layout of x-tap pairs
    (twice the memory); with overlap, 4^3 bricks overlapping by one voxel in x
    (u16, 4/3 of the memory).  The occupancy marks voxels above mark_above (u16
    only; tf_mark_level gives a level a TF allows)."""
    nz, ny, nx = src.shape
    dt = U16_NORM if src.dtype in _U16 else F32
    if edge not in (4, 8) or ((pairs or overlap) and edge != 4) or (pairs and overlap):
        raise ValueError("bricks are 4^3 (plain, pairs or overlapping) or 8^3")
    layout = (LAYOUT_BRICK4_PAIRS if pairs else LAYOUT_BRICK4_OVERLAP if overlap else
              LAYOUT_BRICK8 if edge == 8 else LAYOUT_BRICK4)
    nb, nel, nocc = vr_brick_count_layout(layout, nx, ny, nz)
    if out is None:
        data = torch.empty(nel, dtype=src.dtype, device=src.device)
        occ = torch.empty(nocc, dtype=torch.uint8, device=src.device) if with_occupancy else None
        out = BrickedVolume(data, (nz, ny, nx), occ, layout, mark_above)
    if out.layout != layout:
        raise ValueError("out has a different brick layout")
    out.mark_above = int(mark_above)
    occp = None if out.occupancy is None else _dev(out.occupancy, "occupancy", torch.uint8, nocc)
    _check(lib().vr_brick_volume(_dev(src, "src", (*_U16, torch.float32)), dt, layout, nx, ny, nz,
                                 _dev(out.data, "bricked", src.dtype, nel), occp, int(mark_above),
                                 _stream(stream)))
    return out


def vr_unbrick_volume(bricked, out=None, stream=None):
    """The [nz][ny][nx] volume of a BrickedVolume in VR_LAYOUT_BRICK4 (a new
    tensor, or written into out)."""
    if bricked.layout != LAYOUT_BRICK4:
        raise ValueError("vr_unbrick_volume takes the 4^3 brick layout")
    nz, ny, nx = bricked.shape
    nb, _ = vr_brick_count(nx, ny, nz)
    t = bricked.data
    dt = U16_NORM if t.dtype in _U16 else F32
    if out is None:
        out = torch.empty((nz, ny, nx), dtype=t.dtype, device=t.device)
    _check(lib().vr_unbrick_volume(_dev(t, "bricked", (*_U16, torch.float32), nb * 64), dt, nx, ny, nz,
                                   _dev(out, "out", t.dtype, nx * ny * nz), _stream(stream)))
    return out


def make_volume(data, spacing=(1.0, 1.0, 1.0)):
    """vr_volume for a uint16 (normalised) or float32 tensor [nz][ny][nx], or a BrickedVolume."""
    if isinstance(data, BrickedVolume):
        t, layout, shape, above = data.data, data.layout, data.shape, data.mark_above
        occ = None if data.occupancy is None else _dev(
            data.occupancy, "occupancy", torch.uint8, vr_brick_count_layout(layout, *shape[::-1])[2]).value
    else:
        t, layout, shape, occ, above = data, LAYOUT_LINEAR, data.shape, None, 0
    if t.dtype in _U16:
        dt = U16_NORM
    elif t.dtype == torch.float32:
        dt = F32
    else:
        raise TypeError(f"unsupported volume dtype {t.dtype}")
    nz, ny, nx = shape
    return vr_volume(_dev(t, "volume").value, dt, layout, nx, ny, nz,
                     (C.c_double * 3)(*[float(s) for s in spacing]), occ, above)


def vol_shape(data):
    return data.shape if isinstance(data, BrickedVolume) else tuple(data.shape)


def make_cameras(cams):
    cams = np.asarray(cams, dtype=np.float64).reshape(-1, 11)
    arr = (vr_camera * len(cams))()
    for k, c in enumerate(cams):
        arr[k].eye[:] = [float(x) for x in c[0:3]]
        arr[k].target[:] = [float(x) for x in c[3:6]]
        arr[k].up[:] = [float(x) for x in c[6:9]]
        arr[k].fov_y_deg = float(c[9])
        arr[k].ortho_half_h = float(c[10])
    return arr, len(cams)


def make_opts(width, height, step, ert_eps=2.0 ** -14, bg=(0.0, 0.0, 0.0, 0.0), view_hist=None, flags=0):
    return vr_render_opts(int(width), int(height), float(step), float(ert_eps),
                          (C.c_float * 4)(*[float(b) for b in bg]), view_hist, int(flags))


def vr_raycast(data, tf, cams, width, height, step, spacing=(1.0, 1.0, 1.0), ert_eps=2.0 ** -14,
               bg=(0.0, 0.0, 0.0, 0.0), out=None, samples=None, stream=None, view_hist=None, staged=False):
    """RGBA frames [V][H][W][4] float32; `samples` (int64[2]) accumulates the sample
    counts: [0] samples taken before early termination, [1] samples evaluated;
    `view_hist` (int32 [V][256]) receives the grey-value counts of the frames;
    `staged` selects the depth-window march with LDS staging (VR_RENDER_STAGED)."""
    vol = make_volume(data, spacing)
    ca, nv = make_cameras(cams)
    vh = None if view_hist is None else _dev(view_hist, "view_hist", torch.int32, nv * 256).value
    opts = make_opts(width, height, step, ert_eps, bg, vh, RENDER_STAGED if staged else 0)
    if out is None:
        out = torch.empty((nv, height, width, 4), dtype=torch.float32, device=data.device)
    sp = None if samples is None else _dev(samples, "samples", torch.int64, 2)
    _check(lib().vr_raycast(C.byref(vol), _dev(tf, "tf", torch.float32, 1024), ca, nv,
                            C.byref(opts), _dev(out, "out", torch.float32, nv * height * width * 4),
                            sp, _stream(stream)))
    return out


def vr_frame_entropy(frames, hist=None, entropy=None, best=None, stream=None):
    """Best view of RGBA frames [V][H][W][4] f32 by the entropy of their grey-value
    histograms: -> (best view int32[1], entropies f64[V], counts int32[V][256])."""
    nv, h, w, four = frames.shape
    if four != 4:
        raise ValueError("frames must be [V][H][W][4]")
    if hist is None:
        hist = torch.empty((nv, 256), dtype=torch.int32, device=frames.device)
    if entropy is None:
        entropy = torch.empty(nv, dtype=torch.float64, device=frames.device)
    if best is None:
        best = torch.empty(1, dtype=torch.int32, device=frames.device)
    _check(lib().vr_frame_entropy(_dev(frames, "frames", torch.float32, nv * h * w * 4), nv, w, h,
                                  _dev(hist, "hist", torch.int32, nv * 256),
                                  _dev(entropy, "entropy", torch.float64, nv),
                                  _dev(best, "best", torch.int32, 1), _stream(stream)))
    return best, entropy, hist


def vr_entropy_from_counts(hist, pixels, entropy=None, best=None, stream=None):
    """Entropies and best view from grey-value counts [V][256] of frames of `pixels` pixels."""
    nv = hist.shape[0]
    if entropy is None:
        entropy = torch.empty(nv, dtype=torch.float64, device=hist.device)
    if best is None:
        best = torch.empty(1, dtype=torch.int32, device=hist.device)
    _check(lib().vr_entropy_from_counts(_dev(hist, "hist", torch.int32, nv * 256), nv, int(pixels),
                                        _dev(entropy, "entropy", torch.float64, nv),
                                        _dev(best, "best", torch.int32, 1), _stream(stream)))
    return best, entropy


def vr_raycast_backward(data, tf, cams, width, height, step, rgba_fwd, grad_rgba, grad_density,
                        grad_tf, spacing=(1.0, 1.0, 1.0), ert_eps=2.0 ** -14,
                        bg=(0.0, 0.0, 0.0, 0.0), stream=None, occupancy=None):
    """Adds dLoss/dDensity and dLoss/dTF into grad_density / grad_tf (zero them first).
    data: an f32 [nz][ny][nx] tensor, or its BrickedVolume (4^3 bricks); grad_density
    has the same layout (vr_unbrick_volume brings a bricked one back).
    occupancy: the occupancy grid vr_brick_volume wrote for the same grid, or None
    (with it, runs of samples in empty bricks are not marched)."""
    vol = make_volume(data, spacing)
    if occupancy is not None:
        vol.occupancy = _dev(occupancy, "occupancy", torch.uint8, vr_brick_count(*vol_shape(data)[::-1])[1]).value
    ca, nv = make_cameras(cams)
    opts = make_opts(width, height, step, ert_eps, bg)
    n = nv * height * width * 4
    if isinstance(data, BrickedVolume):
        nz, ny, nx = data.shape
        n_grad = vr_brick_count(nx, ny, nz)[0] * 64
    else:
        n_grad = int(np.prod(vol_shape(data)))
    _check(lib().vr_raycast_backward(
        C.byref(vol), _dev(tf, "tf", torch.float32, 1024), ca, nv, C.byref(opts),
        _dev(rgba_fwd, "rgba_fwd", torch.float32, n), _dev(grad_rgba, "grad_rgba", torch.float32, n),
        _dev(grad_density, "grad_density", torch.float32, n_grad),
        _dev(grad_tf, "grad_tf", torch.float32, 1024), _stream(stream)))
    return grad_density, grad_tf


# ------------------------------------------------------------------ batching
def vr_batch_workspace_size(items, cfg) -> int:
    arr = (vr_batch_item * len(items))(*items)
    n = C.c_int64(0)
    _check(lib().vr_batch_workspace_size(arr, len(items), C.byref(cfg), C.byref(n)))
    return int(n.value)


def vr_batch_plan_create(items, cfg, tf, workspace):
    arr = (vr_batch_item * len(items))(*items)
    plan = C.c_void_p(None)
    _check(lib().vr_batch_plan_create(arr, len(items), C.byref(cfg), _dev(tf, "tf", torch.float32, 1024),
                                      _dev(workspace, "workspace"), workspace.numel() * workspace.element_size(),
                                      C.byref(plan)))
    return plan


def vr_batch_launch(plan, stream=None):
    _check(lib().vr_batch_launch(plan, _stream(stream)))


def vr_batch_capture(plan, stream=None):
    _check(lib().vr_batch_capture(plan, _stream(stream)))


def vr_batch_status(plan):
    st = C.c_uint32(0)
    sm = (C.c_uint64 * 2)()
    _check(lib().vr_batch_status(plan, C.byref(st), sm))
    return int(st.value), (int(sm[0]), int(sm[1]))


def vr_batch_item_outputs(plan, item):
    lv, res, nt = C.c_void_p(None), C.c_void_p(None), C.c_int64(0)
    _check(lib().vr_batch_item_outputs(plan, item, C.byref(lv), C.byref(res), C.byref(nt)))
    return lv.value, res.value, int(nt.value)


def vr_batch_plan_destroy(plan):
    _check(lib().vr_batch_plan_destroy(plan))
