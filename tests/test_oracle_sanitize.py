"""The FP64 oracle ray caster built with AddressSanitizer and UBSan (gcc, host
code only) and run on small volumes whose rays graze, miss and leave through
every face: no sanitizer report, and the frames and sample counts equal those
of the ordinary oracle build bit for bit."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import render as R
from paper_2311_15038_amd import synth

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

pytestmark = pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc is not installed")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("san") / "render_san")
    cmd = ["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-ffp-contract=off", "-o", exe,
           os.path.join(HERE, "sanitize_render_driver.c"), os.path.join(ROOT, "oracle", "render.c"), "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip(f"sanitizer build unavailable: {r.stderr[-300:]}")
    return exe


def _run(exe, tmp, vol, spacing, tf, cams, W, H, step, ert_eps, bg):
    nz, ny, nx = vol.shape
    dt = 0 if vol.dtype == np.uint16 else 1
    cams = np.asarray(cams, dtype=np.float64).reshape(-1, 11)
    inp, outp = os.path.join(tmp, "in.bin"), os.path.join(tmp, "out.bin")
    with open(inp, "wb") as f:
        f.write(np.array([nx, ny, nz, dt, len(cams), W, H], dtype=np.int64).tobytes())
        f.write(np.array([*spacing, step, ert_eps, *bg], dtype=np.float64).tobytes())
        f.write(np.ascontiguousarray(tf, dtype=np.float64).tobytes())
        f.write(cams.tobytes())
        f.write(np.ascontiguousarray(vol).tobytes())
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe, inp, outp], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0 and "runtime error" not in r.stderr and "Sanitizer" not in r.stderr, r.stderr[-2000:]
    raw = open(outp, "rb").read()
    n = len(cams) * H * W * 4
    rgba = np.frombuffer(raw[: 8 * n], dtype=np.float64).reshape(len(cams), H, W, 4)
    rest = np.frombuffer(raw[8 * n:], dtype=np.int64)
    return rgba, rest[: len(cams)], rest[len(cams):].reshape(len(cams), 2)


def _cams(nx, ny, nz):
    tt = synth.turntable_cameras(nx, ny, nz, n_views=3)
    c = np.array([nx / 2, ny / 2, nz / 2])
    extra = [
        [*(c + [0.0, -3.0 * ny, 0.0]), *c, 0, 0, 1, 0.0, 0.6 * max(nx, nz)],     # orthographic, front
        [*(c + [2.0 * nx, 0.0, 0.0]), *(c + [4.0 * nx, 0.0, 0.0]), 0, 0, 1, 40.0, 0.0],   # looks away
        [*(c + [0.0, 0.0, 3.0 * nz]), *c, 0, 1, 0, 75.0, 0.0],                   # straight down z
        [*(c + [nx, ny, 0.5 * nz]), *c, 0, 0, 1, 120.0, 0.0],                    # wide: rays graze the faces
    ]
    return np.concatenate([tt, np.array(extra, dtype=np.float64)])


@pytest.mark.parametrize("shape,dtype,W,H", [((7, 9, 13), np.uint16, 11, 7), ((1, 1, 1), np.uint16, 5, 3),
                                             ((3, 1, 6), np.float32, 9, 4), ((2, 5, 1), np.uint16, 1, 1)])
def test_sanitized_oracle_equals_plain_build(driver, tmp_path, shape, dtype, W, H):
    rng = np.random.default_rng(sum(shape) * 31 + W)
    if dtype == np.uint16:
        vol = rng.integers(0, 65536, size=shape, dtype=np.uint16)
    else:
        vol = rng.random(shape, dtype=np.float32)
    nz, ny, nx = shape
    spacing = (1.0, 1.5, 0.75)
    tf = synth.default_tf(sigma_scale=2.0).astype(np.float64)
    cams = _cams(nx * spacing[0], ny * spacing[1], nz * spacing[2])
    bg = (0.1, 0.2, 0.3, 1.0)
    for ert in (0.0, 2.0 ** -14):
        got, gs, gb = _run(driver, str(tmp_path), vol, spacing, tf, cams, W, H, 0.37, ert, bg)
        ref, rs, rb = R.render(vol, spacing, tf, cams, W, H, 0.37, ert_eps=ert, bg=bg, bounds=True)
        assert np.array_equal(got, ref)
        assert np.array_equal(gs, rs)
        assert np.array_equal(gb, rb)
