"""Benchmark of the preview hot path on one MI355X.

    python bench.py [--steps K] [--warmup W] [--no-cpu] [--no-extras]

One step = one pass of the whole path over the 1024^3 u16 volume resident in
HBM: histogram of the volume and of its first three slices, valley threshold
+ top-slice filter, fused 4-level pyramid, 256^3 -> 4096^2 slicemap atlas,
and 36 perspective turntable frames of 512^2 ray cast from the 512^3 level
(step 0.5).  Prints one JSON line.  `value` is rendered samples per second of
whole-step wall time (reduction included); the reduction's own bandwidth, the
per-kernel times, the forward+backward fit iteration and the oracle's CPU
rate are reported beside it.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0            # MI355X HBM3E, published
FP32_PEAK_TFLOPS = 157.3         # MI355X vector FP32, published
# FP32 operations of one ray-casting sample (FMA = 2): position 6, voxel
# coordinates 6, trilinear fractions 3, seven lerps 21, normalisation 1, TF
# index 2, four TF lerps 12, extinction + exp + alpha 3, compositing 8.
FLOPS_PER_SAMPLE = 62
METRIC = "Gsamples/s ray casting + GB/s reduction vs HBM peak; fwd+bwd, batched vs plain"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _events(n):
    import torch
    return [torch.cuda.Event(enable_timing=True) for _ in range(n)]


def run_gpu(steps, warmup):
    import numpy as np
    import torch

    from paper_2311_15038_amd import pipeline as P
    from paper_2311_15038_amd import synth

    dev = torch.device("cuda:0")
    t0 = time.time()
    vol = synth.make_volume(synth.FULL, dev)
    torch.cuda.synchronize()
    log(f"generated 1024^3 volume in {time.time() - t0:.1f} s")
    pipe = P.PreviewPipeline(vol.shape, P.PreviewConfig(), device=dev)

    # sample count of one step (same every step: deterministic)
    pipe.samples.zero_()
    pipe.step(vol, count=True)
    torch.cuda.synchronize()
    samples = int(pipe.samples[0].item())
    evaluated = int(pipe.samples[1].item())
    for _ in range(warmup):
        pipe.step(vol)
    torch.cuda.synchronize()
    log(f"warmup done ({warmup} steps), {samples} samples per step")

    calls = pipe.calls(vol)
    ev = _events(2)
    k_ev = {name: _events(2 * steps) for name, _ in calls}
    torch.cuda.synchronize()
    ev[0].record()
    for st in range(steps):
        for name, fn in calls:
            k_ev[name][2 * st].record()
            fn()
            k_ev[name][2 * st + 1].record()
    ev[1].record()
    torch.cuda.synchronize()
    total_ms = ev[0].elapsed_time(ev[1])
    per = {k: sum(e[2 * st].elapsed_time(e[2 * st + 1]) for st in range(steps)) / steps
           for k, e in k_ev.items()}
    ms_step = total_ms / steps
    red_ms = sum(per[k] for k in pipe.REDUCTION_CALLS)
    red_bytes = pipe.reduction_bytes()
    T = int(pipe.result[0].item())
    out = {
        "samples_per_step": samples,
        "evaluated_per_step": evaluated,
        "ms_per_step": ms_step,
        "kernel_ms": per,
        "reduction_ms": red_ms,
        "reduction_bytes": red_bytes,
        "threshold": T,
    }
    nz, ny, nx = vol.shape
    vol_b = nx * ny * nz * 2
    lv_b = sum(l.numel() * 2 for l in pipe.levels)
    out["kernel_bytes"] = {"histograms": vol_b + nx * ny * 3 * 2,
                           "pyramid+atlas": vol_b + lv_b + pipe.atlas.numel() * 2,
                           "bricks": 2 * pipe.levels[0].numel() * 2}
    return out, pipe, vol


def run_fwd_bwd(pipe, iters=5):
    """One fit iteration: 16 turntable views at 256^2 of a 256^3 f32 grid
    (spacing 2, step 1 = half its voxel) against renders of the 512^3 level."""
    import torch

    from paper_2311_15038_amd import autograd as VA
    from paper_2311_15038_amd import synth, vr

    dev = pipe.device
    L1 = pipe.levels[0]
    rz, ry, rx = L1.shape
    cams = synth.turntable_cameras(rx, ry, rz, n_views=16)
    tf = pipe.tf
    target = vr.vr_raycast(L1, tf, cams, 256, 256, 0.5)
    dens = (pipe.levels[1].to(torch.float32) / 65535.0).contiguous().requires_grad_(True)
    tfp = tf.clone().requires_grad_(True)
    opt = torch.optim.Adam([dens, tfp], lr=1e-2)

    def it():
        opt.zero_grad(set_to_none=False)
        img = VA.render(dens, tfp, cams, 256, 256, 1.0, (2.0, 2.0, 2.0))
        loss = ((img - target) ** 2).mean()
        loss.backward()
        opt.step()
        return loss

    for _ in range(2):
        it()
    torch.cuda.synchronize()
    e = _events(2)
    e[0].record()
    for _ in range(iters):
        it()
    e[1].record()
    torch.cuda.synchronize()
    it_ms = e[0].elapsed_time(e[1]) / iters
    with torch.no_grad():
        cnt = torch.zeros(2, dtype=torch.int64, device=dev)
        fe = _events(2)
        fe[0].record()
        for _ in range(iters):
            vr.vr_raycast(dens.detach(), tfp.detach(), cams, 256, 256, 1.0, (2.0, 2.0, 2.0))
        fe[1].record()
        vr.vr_raycast(dens.detach(), tfp.detach(), cams, 256, 256, 1.0, (2.0, 2.0, 2.0), samples=cnt)
        torch.cuda.synchronize()
        fwd_ms = fe[0].elapsed_time(fe[1]) / iters
    return {"ms_per_iter": it_ms, "fwd_ms": fwd_ms, "iter_over_fwd": it_ms / fwd_ms,
            "samples_fwd": int(cnt[0].item()), "views": 16, "image": [256, 256], "grid": [256, 256, 256]}


def cpu_baseline(pipe, vol, budget_s=12.0):
    """The oracle, untuned, on a bounded sample of the same step."""
    import numpy as np

    from oracle import reduce as O
    from oracle import render as R
    from paper_2311_15038_amd import synth

    threads = R.threads()
    L1 = synth.to_numpy_u16(pipe.levels[0])
    rz, ry, rx = L1.shape
    cams = pipe.cams
    c = pipe.cfg
    tf = pipe.tf.cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(0)
    n_pix, spent, samples = 256, 0.0, 0
    while spent < budget_s * 0.6:
        pix = np.stack([rng.integers(0, len(cams), n_pix), rng.integers(0, c.height, n_pix),
                        rng.integers(0, c.width, n_pix)], axis=1)
        t0 = time.time()
        _, cnt = R.render_pixels(L1, (1, 1, 1), tf, cams, c.width, c.height, c.step, pix, c.ert_eps)
        spent += time.time() - t0
        samples += cnt
        n_pix *= 2
    render_rate = samples / spent / 1e9
    # reduction oracle on a z-slab of the volume
    slab = synth.to_numpy_u16(vol[:64])
    t0 = time.time()
    H = O.histogram(slab)
    bits = O.keep_bits(O.valley_threshold(H))
    lv = O.pyramid(slab, bits, 4)
    red_s = time.time() - t0
    red_bytes = 2 * slab.nbytes + sum(l.nbytes for l in lv)
    return {"value": render_rate, "unit": "Gsamples/s", "cores": threads, "kind": "oracle",
            "sample": (f"FP64 C oracle (OpenMP, {threads} threads) on {samples} samples of random "
                       f"pixels of the 36 turntable views ({spent:.1f} s); reduction oracle "
                       f"(NumPy, 1 thread) on 64 of the 1024 slices: "
                       f"{red_bytes / red_s / 1e9:.3f} GB/s"),
            "reduction_GB_per_s": red_bytes / red_s / 1e9}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on exactly one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)
    if os.environ.get("WORLD_SIZE", "1") not in ("", "1"):
        print(json.dumps({"error": "single-GPU build; launch without torch.distributed"}))
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)

    res, pipe, vol = run_gpu(args.steps, args.warmup)
    ms = res["ms_per_step"]
    samples = res["samples_per_step"]
    value = samples / (ms * 1e-3) / 1e9
    rc_ms = res["kernel_ms"]["raycast"]
    evaluated = res["evaluated_per_step"]
    # ALU roofline over the samples the kernel evaluates (empty-brick samples are passed over)
    achieved = evaluated * FLOPS_PER_SAMPLE / (rc_ms * 1e-3) / 1e12
    red_gbs = res["reduction_bytes"] / (res["reduction_ms"] * 1e-3) / 1e9
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "Gsamples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32+f32",
        "data": "synthetic (seeded 1024^3 u16 micro-CT phantom, Poisson x64 + Gaussian noise)",
        "config": {"workload": ("1024^3 u16: 65536-bin histograms (volume + top 3 slices), valley "
                                "threshold + top-slice filter, 4-level pyramid, 256^3 -> 4096^2 "
                                "slicemap, 36 x 512^2 perspective turntable of the 512^3 level, "
                                "step 0.5, ERT 2^-14"),
                   "volume": [1024, 1024, 1024], "levels": 4, "views": 36, "image": [512, 512]},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP32_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP32_PEAK_TFLOPS, "traffic": None,
                     "kernel": "raycast_fwd<u16,brick4>", "flops_per_sample": FLOPS_PER_SAMPLE,
                     "samples": "evaluated",
                     "kernel_ms": rc_ms},
        "raycast_Gsamples_per_s": samples / (rc_ms * 1e-3) / 1e9,
        "raycast_evaluated_Gsamples_per_s": evaluated / (rc_ms * 1e-3) / 1e9,
        "samples_per_step": samples,
        "evaluated_per_step": evaluated,
        "reduction": {"ms": res["reduction_ms"], "bytes": res["reduction_bytes"],
                      "GB_per_s": red_gbs, "frac_hbm_peak": red_gbs / HBM_PEAK_GBS,
                      "threshold": res["threshold"]},
        "kernel_ms": res["kernel_ms"],
        "kernel_GB_per_s": {k: b / (res["kernel_ms"][k] * 1e-3) / 1e9
                            for k, b in res["kernel_bytes"].items()},
    }
    if not args.no_extras:
        try:
            fb = run_fwd_bwd(pipe)
            line["fwd_bwd"] = fb
        except Exception as e:  # reported, not hidden
            line["fwd_bwd"] = {"error": repr(e)}
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(pipe, vol)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
