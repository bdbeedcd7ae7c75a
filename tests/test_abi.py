"""The C ABI library loads, exports every function include/vr.h declares, and
rejects bad arguments before touching the device (host logic only)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "vr.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b(vr_\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    from paper_2311_15038_amd import vr
    if not os.path.exists(vr.LIB_PATH):
        from paper_2311_15038_amd import build
        build.build()
    return vr.lib()


def test_header_declares_the_boundary():
    names = _declared()
    for n in ["vr_histogram", "vr_select_threshold", "vr_threshold_downsample", "vr_pack_slicemap",
              "vr_raycast", "vr_raycast_backward", "vr_last_error", "vr_version"]:
        assert n in names, n


def test_library_exports_every_declared_symbol(lib):
    for n in _declared():
        assert hasattr(lib, n), n


def test_version_and_empty_error(lib):
    assert lib.vr_version().decode().startswith("vr ")
    assert lib.vr_last_error().decode() == ""


def test_validation_happens_on_the_host(lib):
    # NULL output, bad dims, bad ranges: rejected before any device work
    assert lib.vr_histogram(None, 4, 4, 4, 0, 4, None, None) == -1
    assert "d_hist" in lib.vr_last_error().decode()
    assert lib.vr_histogram(C.c_void_p(16), 0, 4, 4, 0, 4, C.c_void_p(16), None) == -2
    assert lib.vr_histogram(C.c_void_p(16), 4, 4, 4, 3, 2, C.c_void_p(16), None) == -3
    assert lib.vr_select_threshold(C.c_void_p(16), None, 9, 0, C.c_void_p(16), C.c_void_p(16), None) == -3
    assert lib.vr_select_threshold(C.c_void_p(16), None, 0, 0, C.c_void_p(16), C.c_void_p(16), None) == -3
    ptrs = (C.c_void_p * 9)(*([16] * 9))
    assert lib.vr_threshold_downsample(C.c_void_p(16), 8, 8, 8, None, 9, ptrs, None, None, None) == -3
    assert lib.vr_threshold_downsample(C.c_void_p(16), 8, 8, 8, None, 0, ptrs, None, None, None) == -3
    # levels past the fourth are formed from the level-4 sums: that buffer is required
    assert lib.vr_threshold_downsample(C.c_void_p(16), 8, 8, 8, None, 5, ptrs, None, None, None) == -1
    assert "h_level_sums[3]" in lib.vr_last_error().decode()
    no_s4 = (C.c_void_p * 5)(16, 16, 16, None, 16)
    assert lib.vr_threshold_downsample(C.c_void_p(16), 8, 8, 8, None, 5, ptrs, no_s4, None, None) == -1
    from paper_2311_15038_amd import vr
    spec = vr.vr_atlas_spec(2, 1, 1, 16, 16)       # 1 x 1 tiles cannot hold the 2 slices of level 2
    assert lib.vr_threshold_downsample(C.c_void_p(16), 8, 8, 8, None, 2, ptrs, None, C.byref(spec), None) == -3
    spec = vr.vr_atlas_spec(3, 4, 4, 16, 16)       # level 3 is not produced
    assert lib.vr_threshold_downsample(C.c_void_p(16), 8, 8, 8, None, 2, ptrs, None, C.byref(spec), None) == -3
    assert lib.vr_histogram_with_top(C.c_void_p(16), 4, 4, 4, 5, C.c_void_p(16), C.c_void_p(16), None) == -3
    assert lib.vr_histogram_with_top(C.c_void_p(16), 4, 4, 4, 3, None, C.c_void_p(16), None) == -1
    assert lib.vr_pack_slicemap(C.c_void_p(16), 4, 4, 10, 3, 3, 16, C.c_void_p(16), None) == -3
    assert lib.vr_pack_slicemap(C.c_void_p(16), 4, 4, 9, 3, 3, 12, C.c_void_p(16), None) == -3


def test_raycast_validation_on_the_host(lib):
    from paper_2311_15038_amd import vr, synth
    vol = vr.vr_volume(16, vr.U16_NORM, 0, 8, 8, 8, (C.c_double * 3)(1, 1, 1))
    cams, nv = vr.make_cameras(synth.turntable_cameras(8, 8, 8, n_views=2))
    ok = vr.make_opts(8, 8, 0.5)
    assert lib.vr_raycast(C.byref(vol), C.c_void_p(16), cams, nv, C.byref(ok), None, None, None) == -1
    bad = vr.make_opts(8, 8, -1.0)
    assert lib.vr_raycast(C.byref(vol), C.c_void_p(16), cams, nv, C.byref(bad), C.c_void_p(16), None, None) == -3
    bad = vr.make_opts(0, 8, 0.5)
    assert lib.vr_raycast(C.byref(vol), C.c_void_p(16), cams, nv, C.byref(bad), C.c_void_p(16), None, None) == -2
    vol.dtype = 7
    assert lib.vr_raycast(C.byref(vol), C.c_void_p(16), cams, nv, C.byref(ok), C.c_void_p(16), None, None) == -4
    vol.dtype = vr.U16_NORM
    vol.spacing[1] = 0.0
    assert lib.vr_raycast(C.byref(vol), C.c_void_p(16), cams, nv, C.byref(ok), C.c_void_p(16), None, None) == -3
    vol.spacing[1] = 1.0
    # an occupancy marking level is a u16 value, and 0 for f32 volumes
    vol.occupancy_above = 65536
    assert lib.vr_raycast(C.byref(vol), C.c_void_p(16), cams, nv, C.byref(ok), C.c_void_p(16), None, None) == -3
    vol.occupancy_above, vol.dtype = 3, vr.F32
    assert lib.vr_raycast(C.byref(vol), C.c_void_p(16), cams, nv, C.byref(ok), C.c_void_p(16), None, None) == -3
    assert "occupancy_above" in lib.vr_last_error().decode()
    vol.occupancy_above, vol.dtype = 0, vr.U16_NORM
    # overlapping bricks hold u16 volumes with 32-bit offsets only
    vol.layout, vol.dtype = vr.LAYOUT_BRICK4_OVERLAP, vr.F32
    assert lib.vr_raycast(C.byref(vol), C.c_void_p(16), cams, nv, C.byref(ok), C.c_void_p(16), None, None) == -4
    vol.dtype, vol.nx, vol.ny, vol.nz = vr.U16_NORM, 3 * 1024 + 1, 512, 512   # 1025 x 128 x 128 bricks
    assert lib.vr_raycast(C.byref(vol), C.c_void_p(16), cams, nv, C.byref(ok), C.c_void_p(16), None, None) == -2
    assert "2^24 bricks" in lib.vr_last_error().decode()
    vol.layout, vol.nx, vol.ny, vol.nz = 0, 8, 8, 8
    # the adjoint differentiates f32 grids only
    assert lib.vr_raycast_backward(C.byref(vol), C.c_void_p(16), cams, nv, C.byref(ok), C.c_void_p(16),
                                   C.c_void_p(16), C.c_void_p(16), C.c_void_p(16), None) == -4


def test_brick_validation_on_the_host(lib):
    from paper_2311_15038_amd import vr
    p = C.c_void_p(256)
    assert lib.vr_brick_volume(None, vr.U16_NORM, vr.LAYOUT_BRICK4, 8, 8, 8, p, None, 0, None) == -1
    assert lib.vr_brick_volume(p, 5, vr.LAYOUT_BRICK4, 8, 8, 8, p, None, 0, None) == -4
    assert lib.vr_brick_volume(p, vr.U16_NORM, vr.LAYOUT_LINEAR, 8, 8, 8, p, None, 0, None) == -3
    assert lib.vr_brick_volume(p, vr.U16_NORM, 7, 8, 8, 8, p, None, 0, None) == -3
    assert lib.vr_brick_volume(p, vr.U16_NORM, vr.LAYOUT_BRICK4_PAIRS, 0, 8, 8, p, None, 0, None) == -2
    assert lib.vr_brick_volume(p, vr.U16_NORM, vr.LAYOUT_BRICK4_PAIRS, 8, 8, 8, C.c_void_p(258), None, 0, None) == -3
    # the marking level: u16 values only, and 0 for f32
    assert lib.vr_brick_volume(p, vr.U16_NORM, vr.LAYOUT_BRICK4, 8, 8, 8, p, None, -1, None) == -3
    assert lib.vr_brick_volume(p, vr.U16_NORM, vr.LAYOUT_BRICK4, 8, 8, 8, p, None, 65536, None) == -3
    assert lib.vr_brick_volume(p, vr.F32, vr.LAYOUT_BRICK4, 8, 8, 8, p, None, 1, None) == -3
    assert "mark_above" in lib.vr_last_error().decode()
    assert lib.vr_hollow(None, 8, 8, 8, 1, p, None, None) == -1
    assert lib.vr_hollow(p, 8, 0, 8, 1, C.c_void_p(1 << 20), None, None) == -2
    assert lib.vr_hollow(p, 8, 8, 8, 0, C.c_void_p(1 << 20), None, None) == -3
    assert lib.vr_hollow(p, 8, 8, 8, vr.HOLLOW_MAX_THICKNESS + 1, C.c_void_p(1 << 20), None, None) == -3
    assert lib.vr_hollow(p, 8, 8, 8, 2, C.c_void_p(p.value + 1000), None, None) == -3   # overlap
    assert "overlaps" in lib.vr_last_error().decode()
    assert lib.vr_unbrick_volume(None, vr.F32, 8, 8, 8, p, None) == -1
    assert lib.vr_unbrick_volume(p, 7, 8, 8, 8, p, None) == -4
    assert lib.vr_unbrick_volume(p, vr.U16_NORM, 8, 0, 8, p, None) == -2
    n, o = C.c_int64(0), C.c_int64(0)
    assert lib.vr_brick_count(9, 5, 4, C.byref(n), C.byref(o)) == 0
    # marks, group marks, distance grid and its working bytes
    assert n.value == 3 * 2 * 1 and o.value == 6 + 1 + 6 + 6
    e = C.c_int64(0)
    assert lib.vr_brick_count_layout(vr.LAYOUT_BRICK8, 9, 5, 17, C.byref(n), C.byref(e), C.byref(o)) == 0
    # the bricks, then the apron: one brick layer, one brick row and one brick
    assert n.value == 2 * 1 * 3 and e.value == (6 + 2 * 1 + 2 + 1) * 512 and o.value == 3 * 6 + 1
    assert lib.vr_brick_count_layout(vr.LAYOUT_BRICK4_PAIRS, 9, 5, 4, C.byref(n), C.byref(e), None) == 0
    assert n.value == 6 and e.value == (6 + 3 * 2 + 3 + 1) * 128
    # overlapping 4^3 bricks: brick x serves base taps 3 bx .. 3 bx + 2, (nx - 1) / 3 + 1 of them
    assert lib.vr_brick_count_layout(vr.LAYOUT_BRICK4_OVERLAP, 9, 5, 4, C.byref(n), C.byref(e), C.byref(o)) == 0
    assert n.value == 3 * 2 * 1 and e.value == (6 + 3 * 2 + 3 + 1) * 64 and o.value == 3 * 6 + 1
    assert lib.vr_brick_count_layout(vr.LAYOUT_BRICK4_OVERLAP, 10, 1, 1, C.byref(n), None, None) == 0
    assert n.value == 4
    assert lib.vr_brick_volume(C.c_void_p(256), vr.F32, vr.LAYOUT_BRICK4_OVERLAP, 8, 8, 8, C.c_void_p(256), None, 0,
                               None) == -4
    assert lib.vr_brick_count_layout(vr.LAYOUT_LINEAR, 9, 5, 4, C.byref(n), None, None) == -3
    assert lib.vr_brick_count_layout(vr.LAYOUT_BRICK8, 0, 5, 4, C.byref(n), None, None) == -2


def test_container_validation_on_the_host(lib):
    from paper_2311_15038_amd import vr
    p, b = C.c_void_p(256), C.c_int64(0)
    a256 = lambda n: (n + 255) // 256 * 256  # noqa: E731
    assert lib.vr_container_workspace_size(100, 80, 40, C.byref(b)) == 0
    assert b.value == a256(24) + a256(4 * 41) + a256(4 * 8000) + a256(8 * 8000) + a256(16 * 98 * 78)
    assert lib.vr_container_workspace_size(2, 80, 40, C.byref(b)) == -2          # slice too small
    assert lib.vr_container_workspace_size(8193, 80, 40, C.byref(b)) == -2
    assert lib.vr_container_workspace_size(100, 80, 4097, C.byref(b)) == -3      # radius too large
    need = b.value if lib.vr_container_workspace_size(100, 80, 40, C.byref(b)) == 0 else 0
    ok = lambda **k: lib.vr_find_container(k.get("s", p), 100, 80, k.get("r0", 10), k.get("r1", 40),  # noqa: E731
                                           k.get("sh", 4), k.get("m", 2), k.get("w", p), k.get("wb", need),
                                           k.get("c", p), None)
    assert ok(s=None) == -1 and ok(w=None) == -1 and ok(c=None) == -1
    assert ok(r0=0) == -3 and ok(r0=41) == -3 and ok(sh=17) == -3 and ok(m=-1) == -3
    assert ok(wb=need - 1) == -7
    assert ok(w=C.c_void_p(128)) == -3                                           # unaligned workspace
    # the no-allocation variant: same validation, and the scratch array's size limit
    na = lambda **k: lib.vr_find_container_noalloc(k.get("s", p), k.get("nx", 100), k.get("ny", 80),  # noqa: E731
                                                   k.get("r0", 10), k.get("r1", 40), 4, 2, k.get("c", p), None)
    assert na(s=None) == -1 and na(c=None) == -1 and na(r0=0) == -3 and na(nx=2) == -2
    assert lib.vr_container_workspace_size(1100, 1100, 550, C.byref(b)) == 0
    assert b.value > vr.CONTAINER_SCRATCH_BYTES
    assert na(nx=1100, ny=1100, r0=137, r1=550) == -7
    assert "scratch" in lib.vr_last_error().decode()
    assert lib.vr_container_workspace_size(1024, 1024, 4096, C.byref(b)) == 0
    assert b.value <= vr.CONTAINER_SCRATCH_BYTES                                 # 1024^2 slices fit
    m = re.search(r"#define VR_CONTAINER_SCRATCH_BYTES \((\d+)ll << (\d+)\)", open(HEADER).read())
    assert m and int(m.group(1)) << int(m.group(2)) == vr.CONTAINER_SCRATCH_BYTES
    m = re.search(r"#define VR_BRICK_DIST_CAP (\d+)", open(HEADER).read())
    assert m and int(m.group(1)) == vr.BRICK_DIST_CAP
    assert lib.vr_remove_container(None, 4, 4, 4, p, None) == -1
    assert lib.vr_remove_container(p, 4, 0, 4, p, None) == -2
    assert lib.vr_histogram_in_disc(p, 4, 4, 4, 5, p, p, p, None) == -3
    assert lib.vr_histogram_in_disc(p, 4, 4, 4, 3, None, p, p, None) == -1
    ptrs = (C.c_void_p * 1)(16)
    assert lib.vr_threshold_downsample_in_disc(p, 8, 8, 8, None, None, 1, ptrs, None, None, None) == -1
    assert lib.vr_threshold_downsample_in_disc(p, 8193, 8, 8, None, p, 1, ptrs, None, None, None) == -2


def test_tf_mark_level():
    """The marking level of a TF whose first z knots have zero extinction and finite
    colour: 257 (z - 1) - 1, so that a sample of taps at most that level has a TF
    coordinate below z - 1 (exact arithmetic) and blends knots below z only, and the
    ray caster's reach, floor(V 255 / 65535 (1 + 2^-16)) + 2 knots, stays within z."""
    import math
    import numpy as np
    from paper_2311_15038_amd import vr
    for z in range(0, 257):
        tf = np.ones((256, 4), dtype=np.float32)
        tf[:z, 3] = 0.0
        V = vr.tf_mark_level(tf)
        if z < 2:
            assert V == 0
            continue
        assert V == 257 * (z - 1) - 1 and 0 < V <= 65535
        assert V * 255 < (z - 1) * 65535
        assert min(254, math.floor(V * 255 / 65535 * (1 + 2.0 ** -16))) + 2 <= z
    tf = np.zeros((256, 4), dtype=np.float32)
    tf[5, 0] = np.inf                                 # a colour that is not finite ends the run
    assert vr.tf_mark_level(tf) == 257 * 4 - 1
    tf[0, 3] = 0.5
    assert vr.tf_mark_level(tf) == 0
