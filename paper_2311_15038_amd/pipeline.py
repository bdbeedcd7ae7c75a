"""The preview pipeline for one volume: buffers plus the ordered library calls.

One step, all on one stream with no host synchronisation:
  optionally, the container's circle in the top slice (Section III-B), after
    which every voxel outside it is left out of the steps below,
  histogram of the volume and of its first three slices (Section III-D),
  threshold selection and keep mask on the device (Sections III-A, III-D),
  thresholding fused with the box-filtered pyramid (Section II),
  slicemap atlas of one level (Section III),
  turntable frames ray cast from one level (Section III-C),
  the best view among them by frame entropy (Section III-C, Eq. 2).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import torch

from . import synth, vr


@dataclass
class PreviewConfig:
    n_levels: int = 4
    atlas_level: int = 2            # level packed into the slicemap atlas (0: none)
    render_level: int = 1           # level the frames are rendered from
    n_views: int = 36
    width: int = 512
    height: int = 512
    step: float = 0.5               # world units of the rendered level (its voxel = 1)
    rule: int = vr.RULE_VALLEY
    rule_param: int = 32
    top_slices: int = 3
    fov_deg: float = 60.0
    ortho: bool = False
    ert_eps: float = 2.0 ** -14
    bricked: bool = True            # render from a brick layout
    brick_edge: int = 4             # ... of 4^3 or 8^3 voxels (see tune_bricks)
    overlap: bool = True            # ... 4^3 bricks overlapping by one voxel in x (4/3 of the memory)
    pairs: bool = False             # ... of x-tap pairs (4^3 only; two voxels per load, twice the memory)
    skip_empty: bool = True         # with the brick occupancy (exact)
    mark_by_tf: bool = True         # ... marking voxels above the level the TF leaves empty (exact)
    container: bool = False         # remove the sample container (Section III-B)
    container_radii: tuple | None = None   # (r_min, r_max); None: [min side / 8, min side / 2]
    container_shift: int = 4        # edges: |g|^2 >= 2^-shift of the largest
    container_margin: int = 2       # kept radius = detected radius - margin
    hollow: int = 0                 # data preview (Section II): render the shell of this
                                    # thickness of the rendered level (0: the whole level)


def atlas_tiles(nz: int):
    """Smallest square-ish tile grid holding nz slices."""
    tx = int(math.ceil(math.sqrt(nz)))
    ty = int(math.ceil(nz / tx))
    return tx, ty


class PreviewPipeline:
    def __init__(self, shape, cfg: PreviewConfig, tf: np.ndarray | None = None, device="cuda:0"):
        self.shape = tuple(shape)
        self.cfg = cfg
        dev = torch.device(device)
        self.device = dev
        self.hist = torch.empty(vr.NBINS, dtype=torch.int64, device=dev)
        self.hist_top = torch.empty(vr.NBINS, dtype=torch.int64, device=dev)
        self.result = torch.empty(4, dtype=torch.int32, device=dev)
        self.keep = torch.empty(vr.KEEP_WORDS, dtype=torch.int32, device=dev)
        self.levels = [torch.empty(vr.level_shape(self.shape, k), dtype=torch.uint16, device=dev)
                       for k in range(1, cfg.n_levels + 1)]
        # levels past the fourth are summed from the exact level-4 sums: their buffer
        self._sums = None
        if cfg.n_levels > 4:
            self._sums = [None] * cfg.n_levels
            self._sums[3] = torch.empty(vr.level_shape(self.shape, 4), dtype=torch.int64, device=dev)
        self.tiles, self.atlas = None, None
        if cfg.atlas_level > 0:
            az, ay, ax = self.levels[cfg.atlas_level - 1].shape
            self.tiles = atlas_tiles(az)
            self.atlas = torch.empty((self.tiles[1] * ay, self.tiles[0] * ax), dtype=torch.uint16,
                                     device=dev)
        rz, ry, rx = self.levels[cfg.render_level - 1].shape
        self.render_shape = (rz, ry, rx)
        if cfg.ortho:
            self.cams = synth.front_ortho_camera(rx, ry, rz)
        else:
            self.cams = synth.turntable_cameras(rx, ry, rz, n_views=cfg.n_views, fov_deg=cfg.fov_deg)
        nv = len(self.cams)
        self.frames = torch.empty((nv, cfg.height, cfg.width, 4), dtype=torch.float32, device=dev)
        tf_host = synth.default_tf() if tf is None else tf
        self.tf = torch.from_numpy(tf_host).to(dev)
        # bricks whose voxels are all at or below this level hold only samples of zero
        # extinction under this TF (the ray caster checks the TF again on the device)
        self.mark_above = vr.tf_mark_level(tf_host) if cfg.skip_empty and cfg.mark_by_tf else 0
        self.samples = torch.zeros(2, dtype=torch.int64, device=dev)
        # best-view snapshot of the frames (Section III-C, Eq. 2)
        self.view_hist = torch.empty((nv, 256), dtype=torch.int32, device=dev)
        self.view_entropy = torch.empty(nv, dtype=torch.float64, device=dev)
        self.best_view = torch.empty(1, dtype=torch.int32, device=dev)
        self.circle = self.container_work = None
        if cfg.container:
            nz, ny, nx = self.shape
            self.radii = cfg.container_radii or vr.container_radii(nx, ny)
            self.circle = torch.zeros(vr.CIRCLE_INTS, dtype=torch.int32, device=dev)
            self.container_work = torch.empty(vr.vr_container_workspace_size(nx, ny, self.radii[1]),
                                              dtype=torch.uint8, device=dev)
        self.hollow_level = self.hollow_kept = None
        if cfg.hollow:
            self.hollow_level = torch.empty((rz, ry, rx), dtype=torch.uint16, device=dev)
            self.hollow_kept = torch.zeros(1, dtype=torch.int64, device=dev)
        self.render_vol = None
        # overlapping bricks are 4^3 plain ones (not pairs, not 8^3)
        self.overlap = cfg.overlap and cfg.brick_edge == 4 and not cfg.pairs
        if cfg.bricked:
            layout = (vr.LAYOUT_BRICK4_PAIRS if cfg.pairs else vr.LAYOUT_BRICK4_OVERLAP if self.overlap else
                      vr.LAYOUT_BRICK8 if cfg.brick_edge == 8 else vr.LAYOUT_BRICK4)
            nb, nel, nocc = vr.vr_brick_count_layout(layout, rx, ry, rz)
            occ = torch.empty(nocc, dtype=torch.uint8, device=dev) if cfg.skip_empty else None
            self.render_vol = vr.BrickedVolume(torch.empty(nel, dtype=torch.uint16, device=dev),
                                               (rz, ry, rx), occ, layout)

    def _atlas_arg(self):
        if self.atlas is None:
            return None
        return (self.cfg.atlas_level, self.tiles[0], self.tiles[1], 16, self.atlas)

    def find_container(self, vol, stream=None):
        c = self.cfg
        vr.vr_find_container(vol[0], self.radii[0], self.radii[1], c.container_shift,
                             c.container_margin, self.container_work, self.circle, stream)

    def histograms(self, vol, stream=None):
        c = self.cfg
        if self.circle is not None:
            vr.vr_histogram_in_disc(vol, self.circle, c.top_slices, self.hist, self.hist_top, stream)
        else:
            vr.vr_histogram_with_top(vol, c.top_slices, self.hist, self.hist_top, stream)

    def select(self, stream=None):
        c = self.cfg
        vr.vr_select_threshold(self.hist, self.hist_top, c.rule, c.rule_param, self.result,
                               self.keep, stream)

    def pyramid(self, vol, stream=None):
        vr.vr_threshold_downsample(vol, self.keep, self.cfg.n_levels, self.levels, self._atlas_arg(),
                                   stream, circle=self.circle, sums=self._sums)

    # the reduction half: (the container's circle,) histograms, selection, pyramid
    # with its atlas written in the same pass
    def reduce(self, vol, stream=None):
        if self.circle is not None:
            self.find_container(vol, stream)
        self.histograms(vol, stream)
        self.select(stream)
        self.pyramid(vol, stream)

    def hollow(self, stream=None):
        vr.vr_hollow(self.levels[self.cfg.render_level - 1], self.cfg.hollow, out=self.hollow_level,
                     kept=self.hollow_kept, stream=stream)

    def render(self, stream=None, count=False):
        c = self.cfg
        src = self.levels[c.render_level - 1]
        if self.hollow_level is not None:
            self.hollow(stream)
            src = self.hollow_level
        if self.render_vol is not None:
            vr.vr_brick_volume(src, out=self.render_vol, stream=stream, pairs=self.cfg.pairs,
                               edge=self.cfg.brick_edge, mark_above=self.mark_above, overlap=self.overlap)
            src = self.render_vol
        vr.vr_raycast(src, self.tf, self.cams, c.width, c.height, c.step,
                      ert_eps=c.ert_eps, out=self.frames, samples=self.samples if count else None,
                      stream=stream, view_hist=self.view_hist)

    def snapshot(self, stream=None):
        # the ray caster took the frames' grey-value counts; entropies and the best view from them
        vr.vr_entropy_from_counts(self.view_hist, self.cfg.width * self.cfg.height, self.view_entropy,
                                  self.best_view, stream)

    def step(self, vol, stream=None, count=False):
        self.reduce(vol, stream)
        self.render(stream, count)
        self.snapshot(stream)

    def calls(self, vol, stream=None):
        """The step as named library calls, in order (for per-call timing)."""
        c = self.cfg
        out = [("container", lambda: self.find_container(vol, stream))] if self.circle is not None else []
        out += [
            ("histograms", lambda: self.histograms(vol, stream)),
            ("select", lambda: self.select(stream)),
            ("pyramid+atlas", lambda: self.pyramid(vol, stream)),
        ]
        level = self.levels[c.render_level - 1]
        if self.hollow_level is not None:
            out.append(("hollow", lambda: self.hollow(stream)))
            level = self.hollow_level
        src = level
        if self.render_vol is not None:
            out.append(("bricks", lambda: vr.vr_brick_volume(level, out=self.render_vol, stream=stream,
                                                             pairs=c.pairs, edge=c.brick_edge,
                                                             mark_above=self.mark_above, overlap=self.overlap)))
            src = self.render_vol
        out.append(("raycast", lambda src=src: vr.vr_raycast(src, self.tf, self.cams, c.width, c.height,
                                                             c.step, ert_eps=c.ert_eps, out=self.frames,
                                                             stream=stream, view_hist=self.view_hist)))
        out.append(("best_view", lambda: self.snapshot(stream)))
        return out

    REDUCTION_CALLS = ("histograms", "select", "pyramid+atlas")

    def reduction_bytes(self, separate_steps=False) -> int:
        """Algorithmic HBM bytes of the reduction (histograms, pyramid, atlas): each
        input read once and each output written once.  The atlas is written by the
        pyramid's own pass, so its level is not read again; separate_steps=True
        counts that read too, as a separate packing step would make it."""
        nz, ny, nx = self.shape
        vol = nx * ny * nz * 2
        top = nx * ny * min(self.cfg.top_slices, nz) * 2
        lv = sum(l.numel() * 2 for l in self.levels)
        at_in = at_out = 0
        if self.atlas is not None:
            at_in = self.levels[self.cfg.atlas_level - 1].numel() * 2 if separate_steps else 0
            at_out = self.atlas.numel() * 2
        return vol + top + vol + lv + at_in + at_out


# Brick layouts the tuner chooses from: 4^3 bricks overlapping by one voxel in
# x, plain 4^3 bricks, 8^3 bricks.
BRICK_CHOICES = {"4o": dict(brick_edge=4, overlap=True), "4": dict(brick_edge=4, overlap=False),
                 "8": dict(brick_edge=8, overlap=False)}
BRICK_LAYOUT_NAMES = {"4o": "brick4_overlap", "4": "brick4", "8": "brick8"}


def tune_bricks(pipe: PreviewPipeline, reps: int = 3, use_cache: bool = True, log=None):
    """Pick the brick layout of the rendered level for this pipeline (a key of
    BRICK_CHOICES): times the brick copy plus the frames for each on the
    pipeline's own level (run a step or `reduce` first) with HIP events, and
    keeps the fastest.  Results are cached beside the batch tuner's, keyed by GPU
    architecture, level shape, frame size and views.  Returns
    (choice, {choice: ms}); PreviewConfig(**BRICK_CHOICES[choice]) applies it."""
    import json
    import os

    from . import batch as _batch

    c = pipe.cfg
    level = pipe.levels[c.render_level - 1]
    arch = torch.cuda.get_device_properties(level.device).gcnArchName.split(":")[0]
    key = f"{arch}|single-layout|{'x'.join(map(str, level.shape))}|{c.width}x{c.height}x{len(pipe.cams)}"
    path = _batch._cache_path()
    cache = {}
    if use_cache and os.path.exists(path):
        try:
            with open(path) as f:
                cache = json.load(f)
        except (OSError, ValueError):
            cache = {}
    if use_cache and cache.get(key) in BRICK_CHOICES:
        return cache[key], {}
    times = {}
    for choice, kw in BRICK_CHOICES.items():
        bv = vr.vr_brick_volume(level, edge=kw["brick_edge"], overlap=kw["overlap"], mark_above=pipe.mark_above)
        out = torch.empty_like(pipe.frames)

        def run():
            vr.vr_brick_volume(level, out=bv, edge=kw["brick_edge"], overlap=kw["overlap"],
                               mark_above=pipe.mark_above)
            vr.vr_raycast(bv, pipe.tf, pipe.cams, c.width, c.height, c.step, ert_eps=c.ert_eps, out=out)

        run()
        torch.cuda.synchronize()
        best = float("inf")
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            run()
            e1.record()
            torch.cuda.synchronize()
            best = min(best, e0.elapsed_time(e1))
        times[choice] = best
        if log:
            log(f"bricks {choice}: {best:.3f} ms")
        del bv, out
    choice = min(times, key=times.get)
    if use_cache:
        cache[key] = choice
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            with open(path, "w") as f:
                json.dump(cache, f, indent=1)
        except OSError:
            pass
    return choice, times
