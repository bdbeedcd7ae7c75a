"""Many volumes x many views in one launch (a persistent kernel for the
reduction and brick phases, then one render kernel for every item's views),
with a tuner for its launch shape.

BatchPreview wraps the vr_batch_* entry points: it lays out one workspace for
every item (histograms, masks, level 1, bricks, occupancy, task table), builds
the plan, optionally captures the launch into a HIP graph, and exposes the
per-item outputs as tensor views of the workspace.

tune() times candidate render tiles (pixels per wave, waves per task), brick
sizes (4^3 or 8^3 voxels) and task sizes on the actual batch with HIP events
and keeps the fastest; results are cached in a JSON file keyed by GPU
architecture, a coarse size bucket of the batch and the frame size.
"""
from __future__ import annotations

import ctypes as C
import json
import math
import os

import numpy as np
import torch

from . import synth, vr

DEFAULTS = dict(wave_w=8, wave_h=8, waves_x=4, hist_task_voxels=4 << 20, down_tiles_per_task=16,
                slabs_per_task=32, brick_edge=4)

RENDER_TILES = [(8, 8, 4), (8, 8, 2), (8, 8, 8), (16, 4, 2), (16, 4, 4), (4, 16, 8), (4, 16, 4)]
BRICK_EDGES = [4, 8]
TASK_SIZES = [(4 << 20, 16, 32), (1 << 20, 8, 16), (16 << 20, 32, 64), (4 << 20, 32, 32), (4 << 20, 64, 64)]


def _cfg(width, height, step, ert_eps, bg, rule, rule_param, top_slices, t):
    return vr.vr_batch_config(int(width), int(height), float(step), float(ert_eps),
                              (C.c_float * 4)(*[float(b) for b in bg]), int(rule), int(rule_param),
                              int(top_slices), int(t["wave_w"]), int(t["wave_h"]), int(t["waves_x"]),
                              int(t["hist_task_voxels"]), int(t["down_tiles_per_task"]),
                              int(t["slabs_per_task"]), 1, int(t.get("brick_edge", 4)))


class BatchPreview:
    """Reduction + level-1 bricks + turntable frames for a list of u16 volumes."""

    def __init__(self, volumes, n_views=12, width=256, height=256, step=0.5, tf=None,
                 rule=vr.RULE_VALLEY, rule_param=32, top_slices=3, ert_eps=2.0 ** -14,
                 bg=(0.0, 0.0, 0.0, 0.0), tuning=None, workspace=None):
        self.volumes = list(volumes)
        dev = self.volumes[0].device
        self.device = dev
        self.width, self.height, self.n_views = width, height, n_views
        self.tuning = dict(DEFAULTS, **(tuning or {}))
        self.tf = torch.from_numpy(synth.default_tf() if tf is None else tf).to(dev)
        self.cams = []
        self.frames = []
        self._items = []
        for v in self.volumes:
            nz, ny, nx = v.shape
            lz, ly, lx = vr.level_shape((nz, ny, nx), 1)
            cams = synth.turntable_cameras(lx, ly, lz, n_views=n_views)
            cam_arr, _ = vr.make_cameras(cams)
            self.cams.append((cams, cam_arr))
            fr = torch.empty((n_views, height, width, 4), dtype=torch.float32, device=dev)
            self.frames.append(fr)
            self._items.append(vr.vr_batch_item(
                vr._dev(v, "volume", vr._U16).value, nx, ny, nz, (C.c_double * 3)(1.0, 1.0, 1.0),
                n_views, C.cast(cam_arr, C.c_void_p), fr.data_ptr()))
        self._args = (width, height, step, ert_eps, bg, rule, rule_param, top_slices)
        self.cfg = _cfg(*self._args, self.tuning)
        need = vr.vr_batch_workspace_size(self._items, self.cfg)
        if workspace is None or workspace.numel() < need:
            workspace = torch.empty(need, dtype=torch.uint8, device=dev)
        self.workspace = workspace
        self.plan = vr.vr_batch_plan_create(self._items, self.cfg, self.tf, self.workspace)
        self.captured = False
        self.stream = torch.cuda.Stream(device=dev)

    def capture(self):
        """Capture the launch (both kernels) into a HIP graph (replayed by launch())."""
        with torch.cuda.stream(self.stream):
            vr.vr_batch_capture(self.plan, self.stream)
        self.captured = True

    def launch(self, stream=None):
        vr.vr_batch_launch(self.plan, stream)

    def status(self):
        return vr.vr_batch_status(self.plan)

    def _view(self, ptr, nbytes):
        off = ptr - self.workspace.data_ptr()
        assert 0 <= off and off + nbytes <= self.workspace.numel()
        return self.workspace[off:off + nbytes]

    def level1(self, i):
        lv, _, _ = vr.vr_batch_item_outputs(self.plan, i)
        shape = vr.level_shape(tuple(self.volumes[i].shape), 1)
        n = int(np.prod(shape))
        return self._view(lv, 2 * n).view(torch.int16).view(torch.uint16).view(shape)

    def result(self, i):
        _, res, _ = vr.vr_batch_item_outputs(self.plan, i)
        return self._view(res, 16).view(torch.int32)

    def n_tasks(self):
        return vr.vr_batch_item_outputs(self.plan, 0)[2]

    def close(self):
        if self.plan is not None:
            vr.vr_batch_plan_destroy(self.plan)
            self.plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ tuner
def _cache_path():
    return os.environ.get("VR_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "vr_autotune.json"))


def _key(volumes, width, height, n_views):
    arch = torch.cuda.get_device_properties(volumes[0].device).gcnArchName.split(":")[0]
    vox = sum(v.numel() for v in volumes)
    return f"{arch}|n{len(volumes)}|vox2^{int(math.log2(max(vox, 1)))}|{width}x{height}x{n_views}"


def _time(batch, reps=3):
    batch.launch()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * reps)]
    for r in range(reps):
        ev[2 * r].record()
        batch.launch()
        ev[2 * r + 1].record()
    torch.cuda.synchronize()
    return sorted(ev[2 * r].elapsed_time(ev[2 * r + 1]) for r in range(reps))[reps // 2]


def tune(volumes, n_views=12, width=256, height=256, use_cache=True, log=None, **kw):
    """Pick the render tile and task sizes for this batch; returns (tuning, timings)."""
    key = _key(volumes, width, height, n_views)
    path = _cache_path()
    cache = {}
    if use_cache and os.path.exists(path):
        try:
            with open(path) as f:
                cache = json.load(f)
        except (OSError, ValueError):
            cache = {}
    if use_cache and key in cache:
        return cache[key], {}
    timings = {}                  # configuration -> fastest time seen (ms), status-0 runs only
    best = dict(DEFAULTS)
    ws = None
    # stage 1: render tile shape; stage 2: brick size; stage 3: task sizes, each with the best so far
    for stage in range(3):
        if stage == 0:
            cands = [dict(best, wave_w=a, wave_h=b, waves_x=c) for a, b, c in RENDER_TILES]
        elif stage == 1:
            cands = [dict(best, brick_edge=e) for e in BRICK_EDGES]
        else:
            cands = [dict(best, hist_task_voxels=h, down_tiles_per_task=d, slabs_per_task=s)
                     for h, d, s in TASK_SIZES]
        for t in cands:
            b = BatchPreview(volumes, n_views, width, height, tuning=t, workspace=ws, **kw)
            ws = b.workspace
            ms = _time(b)
            st, _ = b.status()
            b.close()
            name = json.dumps(t, sort_keys=True)
            if log:
                log(f"tune {t}: {ms:.3f} ms status={st}")
            if st == 0:
                timings[name] = min(ms, timings.get(name, float("inf")))
        if timings:
            best = json.loads(min(timings, key=timings.get))
    if use_cache:
        cache[key] = best
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            with open(path, "w") as f:
                json.dump(cache, f, indent=1)
        except OSError:
            pass
    return best, timings
