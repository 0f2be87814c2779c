#!/usr/bin/env python3
"""Benchmark of the PlenOctree renderer on one MI355X.

Workload: the depth-9 Gaussian-blob surface-band tree (~2.9M leaves, SH
degree 3, sigma ~ lognormal(2, 1), SH ~ N(0, 0.5^2)), 200 camera poses
area-uniform on the upper hemisphere at radius 4 looking at the origin,
800x800 pixels, 40 degree horizontal field of view, white background, early
stop at T < 1e-4.  A step is one 800x800 frame: one render_camera call over
all 640,000 rays, i.e. the render pass of five launches (the walk of every
ray, the chunks and sub-chunks of the long walks, the join, and the clearing
of the queue counters).  Inputs are resident in HBM before timing; the image
stays on the device.  The one-pass render of the same frames (one launch,
every ray walked to its end by one lane) is timed beside it.

Prints one JSON line: FPS of the float32 tree (headline value), Msamples/s,
the float16-leaf form, a roofline entry for the render kernel and the FP64
oracle's throughput on the host cores as the CPU baseline.  Further legs: the
optimisation step (differentiation), serving, the viewer outputs, the
visibility filter, the colour-basis sweep and codebook leaves.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "800x800 FPS + Msamples/s, fp32 vs fp16 leaves; served p50/p99 ms; HBM GB/s"
HBM_PEAK_GBPS = 8000.0
W = H = 800
N_POSES = 200
STOP_T = 1e-4


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "render_camera_depth9_800x800_hbm_traffic.md")
TRAIN_TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "train_step_depth8_65536rays_hbm_traffic.md")
KERNEL_SRC = [os.path.join(ROOT, "paper_2103_14024_amd", "csrc", f) for f in ("po_kernels.hip", "po_internal.h")]


def kernel_hash() -> str:
    """First 16 hex digits of the SHA-256 of the kernel source and the
    internal header that holds its tuning constants."""
    import hashlib

    h = hashlib.sha256()
    for src in KERNEL_SRC:
        with open(src, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def counter_traffic(dtype: str, profile: str = TRAFFIC_PROFILE, key: str = "hbm_bytes_per_frame_"):
    """HBM bytes per frame of the float32/float16 render pass (its five
    launches), or with key "hbm_bytes_per_step_" and dtype "train" per
    optimisation step, from a committed rocprofv3 counter summary
    (FETCH_SIZE and WRITE_SIZE, scaled by a plain copy), or None when the
    kernel source changed since."""
    try:
        with open(profile) as f:
            text = f.read()
    except OSError:
        return None
    import re

    h = re.search(r"kernel_source_sha256_16 = `([0-9a-f]+)`", text)
    if h is None or h.group(1) != kernel_hash():
        return None
    vals = dict(re.findall(r"(hbm_bytes_per_\w+) = `(\d+)`", text))
    v = vals.get(key + dtype)
    return float(v) if v else None


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def record_bytes(tree) -> int:
    """Bytes one sample gathers: the density plus the 3K SH coefficients."""
    es = 4 if tree.dtype == 0 else 2
    return es * (1 + 3 * tree.K)


def timed_poses(steps: int, n: int = N_POSES) -> list:
    """Pose of each timed frame: strided over all n poses (every pose once
    when steps == n)."""
    return [(i * n) // steps for i in range(steps)]


def measure(po, tree, cams, steps, warmup, stream, aux_pass=True):
    import torch

    img = torch.empty((H, W, 3), dtype=torch.float32, device="cuda")
    order = timed_poses(steps, len(cams))
    poses = sorted(set(order))
    # per-pose unit counts of the walk (samples, cells, child-entry reads) and
    # lane efficiency of the one-pass walk, outside the timed region
    aux = torch.empty((H, W, po.AUX_WIDTH), dtype=torch.float32, device="cuda")
    stats, wave_iters = {}, []
    for p in (poses if aux_pass else []):
        stats[p] = po.traversal_stats(tree, cams[p], stop_T=STOP_T, stream=stream)
        po.render_camera(tree, cams[p], stop_T=STOP_T, aux=True, out=img, aux_out=aux, stream=stream, one_pass=True)
        a = aux.view(-1, po.AUX_WIDTH).double().sum(0).cpu()  # counts above 2^24: sum in float64
        # the aux output of the one-pass render counts the same samples and cells
        assert int(a[po.AUX_SAMPLES]) == stats[p]["samples"] and int(a[po.AUX_STEPS]) == stats[p]["cells"], p
        # SIMD efficiency of the traversal loop: a wave (8x8 pixels) runs as
        # many iterations as its slowest lane
        st = aux[..., po.AUX_STEPS].view(H // 8, 8, W // 8, 8).amax(dim=(1, 3))
        wave_iters.append(float(st.double().sum()) * 64)
    for i in range(warmup):
        po.render_camera(tree, cams[i % len(cams)], stop_T=STOP_T, out=img, stream=stream)
    torch.cuda.synchronize()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(stream):
        t0.record(stream)
        for i in range(steps):
            po.render_camera(tree, cams[order[i]], stop_T=STOP_T, out=img, stream=stream)
        t1.record(stream)
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1)
    rays = steps * W * H
    if not aux_pass:
        return dict(ms=ms, ms_per_step=ms / steps, fps=steps / (ms * 1e-3), mrays_per_s=rays / (ms * 1e3),
                    poses_timed=len(poses))
    n_samples = sum(stats[p]["samples"] for p in order)
    n_cells = sum(stats[p]["cells"] for p in order)
    n_loads = sum(stats[p]["node_loads"] for p in order)
    lane_eff = sum(stats[p]["cells"] for p in poses) / sum(wave_iters)
    rec = record_bytes(tree)
    alg_bytes = n_samples * rec + n_loads * 4 + rays * 12
    return dict(ms=ms, ms_per_step=ms / steps, fps=steps / (ms * 1e-3), msamples_per_s=n_samples / (ms * 1e3),
                mrays_per_s=rays / (ms * 1e3), samples_per_ray=n_samples / rays, steps_per_ray=n_cells / rays,
                node_loads_per_ray=n_loads / rays, alg_gbps=alg_bytes / (ms * 1e-3) / 1e9,
                alg_bytes_per_launch=alg_bytes / steps,
                alg_bytes_split={"records": n_samples * rec / steps, "child_entries": n_loads * 4 / steps,
                                 "rays": rays * 12 / steps},
                lane_efficiency=lane_eff, poses_timed=len(poses))


def measure_one_pass(po, tree, cams, steps, warmup, stream):
    """The same frames rendered in one pass (a single-job batch: one launch,
    one lane per ray walking it to its end)."""
    import torch

    img = torch.empty((H, W, 3), dtype=torch.float32, device="cuda")
    jobs = [[po.Job(tree, cam, img, stop_T=STOP_T, one_pass=True)] for cam in cams]
    order = timed_poses(steps, len(cams))
    for i in range(warmup):
        po.render_batch(jobs[i % len(cams)], stream=stream)
    torch.cuda.synchronize()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(stream):
        t0.record(stream)
        for i in range(steps):
            po.render_batch(jobs[order[i]], stream=stream)
        t1.record(stream)
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1)
    return {"fps": round(steps / (ms * 1e-3), 2), "ms_per_step": round(ms / steps, 4)}


def measure_end_to_end(po, tree, cams, steps, warmup, stream):
    """Frames delivered to the host: each render followed by the copy of its
    800x800x3 float32 image into pinned host memory.  "serial" copies on the
    render stream (render, copy, render, ...); "overlapped" copies on a second
    stream from two image buffers, so that a frame's copy runs beside the next
    frame's render.  Not the headline: the boundary takes device buffers."""
    import torch

    imgs = [torch.empty((H, W, 3), dtype=torch.float32, device="cuda") for _ in range(2)]
    hosts = [torch.empty((H, W, 3), dtype=torch.float32, pin_memory=True) for _ in range(2)]
    order = timed_poses(steps, len(cams))
    copy_stream = torch.cuda.Stream()
    res = {}
    for mode in ("serial", "overlapped"):
        for rep in range(2):  # the first pass warms up
            n = warmup if rep == 0 else steps
            torch.cuda.synchronize()
            t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            done = [None, None]
            t0.record(stream)
            for i in range(n):
                k = i % 2 if mode == "overlapped" else 0
                if done[k] is not None:
                    stream.wait_event(done[k])
                po.render_camera(tree, cams[order[i % len(order)]], stop_T=STOP_T, out=imgs[k], stream=stream)
                if mode == "serial":
                    with torch.cuda.stream(stream):
                        hosts[0].copy_(imgs[0], non_blocking=True)
                    continue
                ready = torch.cuda.Event()
                ready.record(stream)
                copy_stream.wait_event(ready)
                with torch.cuda.stream(copy_stream):
                    hosts[k].copy_(imgs[k], non_blocking=True)
                done[k] = torch.cuda.Event()
                done[k].record(copy_stream)
            for e in done:
                if e is not None:
                    stream.wait_event(e)
            t1.record(stream)
            torch.cuda.synchronize()
        ms = t0.elapsed_time(t1)
        res[mode] = {"fps": round(steps / (ms * 1e-3), 2), "ms_per_step": round(ms / steps, 4)}
    res["bytes_per_frame"] = H * W * 3 * 4
    return res


ERR_POSES = list(range(0, N_POSES, 20))   # poses whose frames the oracle renders (error and CPU baseline)


def gpu_frames(po, tree, cams, poses):
    """Host copies of the render_camera images of the given poses."""
    out = {}
    for p in poses:
        out[p] = po.render_camera(tree, cams[p], stop_T=STOP_T).cpu().numpy()
    return out


def _err(a, b):
    e = np.abs(np.asarray(a, np.float64) - np.asarray(b, np.float64)).reshape(-1, 3)
    return {"max": [round(float(v), 8) for v in e.max(0)], "mean": [float("%.3e" % v) for v in e.mean(0)]}


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(scene, poses, frames32, frames16, budget_s=12.0, min_frames=5):
    """The FP64 oracle on the host cores, on a bounded sample of the same
    workload: whole 800x800 frames of the poses in ERR_POSES (every 20th
    pose), then of the other poses, until ~budget_s of work and at least
    min_frames frames; scaled to frames per second.  The ERR_POSES frames give the per-channel error of
    the GPU's float32 and float16 renders (frames32, frames16: host images of
    those poses), and an oracle render of the float16-decoded tree on sampled
    pixels gives the float16 form's parity on its own values."""
    import oracle
    from paper_2103_14024_amd import scenes

    t = oracle.OracleTree(scene["depth"], scene["sh_degree"], scene["center"], scene["half"], scene["cells"],
                          scene["sigma"], scene["sh"])
    fx, fy, cx, cy = scenes.intrinsics(W, H, 40.0)
    f32 = [float(np.float32(v)) for v in (fx, fy, cx, cy)]
    n, dt, timed = 0, 0.0, []
    refs = {}
    # the error poses first, then the other poses until the budget
    order = list(ERR_POSES) + [p for p in range(len(poses)) if p not in ERR_POSES]
    for p in order:
        if p not in ERR_POSES and dt >= budget_s and len(timed) >= min_frames:
            break
        o, d = oracle.camera_rays(np.asarray(poses[p], np.float32).astype(np.float64), W, H, *f32)
        t0 = time.perf_counter()
        rgb, _, _, _ = t.render_rays(o, d, gamma=STOP_T)
        dt += time.perf_counter() - t0
        n += len(o)
        timed.append(p)
        if p in ERR_POSES:
            refs[p] = rgb.reshape(H, W, 3)
    rays_per_s = n / dt
    base = {"value": rays_per_s / (W * H), "unit": "FPS", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"{len(timed)} whole 800x800 frames of the same scene (every 20th of the 200 poses, then "
                      f"the others in order), {dt:.1f} s of FP64 rendering, {rays_per_s / 1e6:.2f} Mrays/s"}
    # one core: rows 320-479 (the middle of the image) of the first error pose
    threads = oracle.num_threads()
    o, d = oracle.camera_rays(np.asarray(poses[ERR_POSES[0]], np.float32).astype(np.float64), W, H, *f32)
    oracle.set_num_threads(1)
    try:
        t0 = time.perf_counter()
        t.render_rays(o[320 * W:480 * W], d[320 * W:480 * W], gamma=STOP_T)
        dt1 = time.perf_counter() - t0
    finally:
        oracle.set_num_threads(threads)
    base["single_core"] = {"mrays_per_s": round(160 * W / dt1 / 1e6, 4), "fps": round(160 * W / dt1 / (W * H), 4),
                           "sample": f"rows 320-479 of pose {ERR_POSES[0]}, {dt1:.2f} s"}
    base["nproc"] = len(os.sched_getaffinity(0))
    base["cpu_model"] = _cpu_model()
    done = list(ERR_POSES)
    ref = np.stack([refs[p] for p in done])
    err = {"poses": done, "pixels": int(ref.size // 3),
           "f32_vs_oracle": _err(np.stack([frames32[p] for p in done]), ref)}
    if frames16:
        err["f16_vs_oracle_f32_values"] = _err(np.stack([frames16[p] for p in done]), ref)
        # parity on the float16 values: the oracle on the decoded tree, 20000
        # sampled pixels per frame
        sig16 = np.asarray(scene["sigma"], np.float32).astype(np.float16).astype(np.float64)
        sh16 = np.asarray(scene["sh"], np.float32).astype(np.float16).astype(np.float64)
        t16 = oracle.OracleTree(scene["depth"], scene["sh_degree"], scene["center"], scene["half"], scene["cells"],
                                sig16, sh16)
        rng = np.random.default_rng(0)
        got, want = [], []
        for p in done:
            idx = rng.choice(W * H, 20000, replace=False)
            o, d = oracle.camera_rays(np.asarray(poses[p], np.float32).astype(np.float64), W, H, *f32)
            want.append(t16.render_rays(o[idx], d[idx], gamma=STOP_T)[0])
            got.append(frames16[p].reshape(-1, 3)[idx])
        err["f16_vs_oracle_f16_values"] = dict(_err(np.concatenate(got), np.concatenate(want)),
                                                pixels=int(sum(len(g) for g in got)))
    return base, err


def train_leg(po, scenes, steps=100, warmup=5, fit_steps=300, lr=1e7, batch=65536, psnr=True):
    """Differentiation workload: depth-8 blob tree (SH degree 2, float32),
    targets = 100 renders of 400x400 from the ground-truth tree, training
    from a copy perturbed by N(0, 0.3^2), SGD on random batches of 65536
    rays.  Times full optimisation steps (batch gather, forward, loss
    gradient, backward with atomics, SGD) with HIP events and reports the
    dataset PSNR before and after `fit_steps` steps.

    Roofline of a step, algorithmic bytes: forward and backward each read
    every sample's record (4 (1 + 3K) B) and every child entry of the walk
    (4 B); the backward adds 1 + 3K float atomics per sample (a read and a
    write of 4 B each); rays move 36 B in and 12 B out of the forward, 36 B
    through the loss gradient, 48 B into the backward and 72 B through the
    batch gather; SGD reads and writes the parameters and the gradients of
    every leaf (16 B per value).  Samples and child-entry reads are counted
    on the batches of the warm-up steps (outside the timed region)."""
    import torch

    gt = scenes.scene_train()
    tgt = po.Tree.from_scene(gt)
    fx, fy, cx, cy = scenes.intrinsics(400, 400, 40.0)
    cams = [po.Camera(p, 400, 400, fx, fy, cx, cy) for p in scenes.hemisphere_poses(100, 4.0, 5)]
    o, d, t = po.optim.training_set(tgt, cams)
    del tgt
    sig, sh = scenes.perturb(gt["sigma"], gt["sh"], 0.3, 7)
    tree = po.Tree.from_cells(gt["depth"], gt["sh_degree"], gt["cells"], sig, sh)
    m0 = po.optim.dataset_mse(tree, o, d, t) if psnr else float("nan")
    tr = po.Trainer(tree, o, d, t, lr_sigma=lr, lr_sh=lr, batch=batch, seed=1)
    st = {"samples": 0, "node_loads": 0, "cells": 0}
    warmup = max(1, warmup)
    for _ in range(warmup):
        tr.step()
        c = po.traversal_stats(tree, origins=tr.bo, dirs=tr.bd, stop_T=tr.stop_T)
        for k in st:
            st[k] += c[k] / warmup
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        tr.step()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    for _ in range(max(0, fit_steps - steps - warmup)):
        tr.step()
    m1 = po.optim.dataset_mse(tree, o, d, t) if psnr else float("nan")
    K = tree.K
    rec = 4 * (1 + 3 * K)
    walk = st["samples"] * rec + st["node_loads"] * 4
    parts = {"forward": walk + batch * 48, "loss_grad": batch * 36,
             "backward": walk + st["samples"] * (1 + 3 * K) * 8 + batch * 48, "batch_gather": batch * 72,
             "sgd": tree.n_leaves * (1 + tree.stride) * 16}
    alg = sum(parts.values())
    gbps = alg / (ms * 1e-3) / 1e9
    tb = counter_traffic("train", TRAIN_TRAFFIC_PROFILE, "hbm_bytes_per_step_")
    return {"workload": "depth-8 blob band (%d leaves), SH degree 2, fp32, 100x400x400 targets, batch %d, "
                        "SGD lr %g" % (len(gt["cells"]), batch, lr),
            "ms_per_step": round(ms, 4), "mrays_per_s": round(batch / ms / 1e3, 2),
            "samples_per_ray": round(st["samples"] / batch, 3), "cells_per_ray": round(st["cells"] / batch, 2),
            "child_entry_reads_per_ray": round(st["node_loads"] / batch, 2),
            "roofline": {"bound": "hbm", "achieved": round(gbps, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                         "frac": round(gbps / HBM_PEAK_GBPS, 4),
                         "traffic": None if tb is None else round(tb / (ms * 1e-3) / 1e9, 1),
                         "hbm_bytes_per_step": None if tb is None else int(tb), "alg_bytes_per_step": int(alg),
                         "alg_bytes_per_step_parts": {k: int(v) for k, v in parts.items()},
                         "atomics_per_step": int(st["samples"] * (1 + 3 * K))},
            "psnr_start": round(po.psnr(m0), 2) if psnr else None, "psnr_after": round(po.psnr(m1), 2) if psnr else None,
            "steps_fitted": fit_steps,
            "paper_context": "about 3M rays/s on a Tesla V100 (NeRF-synthetic)"}


def serve_leg(po, scenes, rates=(50, 100, 200, 350, 500, 1000, 1500, 2000), n_requests=2000, budget_mb=1024):
    """Serving workload: four float16 scenes resident in HBM (depth 8/9/9/10,
    SH degree 2/3/2/3), Poisson arrivals at each rate, resolutions uniform
    over 256^2, 512^2, 800^2, 1280x720 and 1920x1080, random upper-hemisphere
    poses, outputs admitted against an HBM budget.  Reports p50/p99 latency
    (arrival to completion on the GPU clock) and throughput per rate."""
    from paper_2103_14024_amd import server

    t0 = time.perf_counter()
    sc = scenes.serve_scenes()
    trees = [po.Tree.from_scene(s, dtype="f16") for s in sc]
    log(f"serve: scenes {[len(s['cells']) for s in sc]} leaves in {time.perf_counter() - t0:.1f} s")
    srv = server.Server(trees, budget_bytes=budget_mb << 20, max_active=64, chunk_tiles=256, launch_tiles=2048,
                        streams=3, max_inflight=4)
    # warm up every kernel variant
    srv.run(server.poisson_requests(20, 1000.0, len(trees), seed=99))
    per_rate = {}
    for k, rate in enumerate(rates):
        st = srv.run(server.poisson_requests(n_requests, float(rate), len(trees), seed=100 + k))
        per_rate[str(rate)] = st.summary()
        log(f"serve {rate} req/s: {per_rate[str(rate)]}")
    return {"workload": "4 resident fp16 scenes (leaves %s), Poisson arrivals, mixed resolutions, "
                        "%d requests per rate, %d MB output budget" % ([len(s["cells"]) for s in sc], n_requests,
                                                                      budget_mb),
            "by_rate": per_rate}


def _time_frames(po, tree, cams, n, **kw):
    """ms per frame of render_camera over n frames (HIP events, after 3 warm-up frames)."""
    import torch

    img = torch.empty((cams[0].height, cams[0].width, 3), dtype=torch.float32, device="cuda")
    aux = None
    if kw.get("aux"):
        aux = torch.empty((cams[0].height, cams[0].width, po.AUX_WIDTH), dtype=torch.float32, device="cuda")
    for i in range(3):
        po.render_camera(tree, cams[i % len(cams)], stop_T=STOP_T, out=img, aux_out=aux, **kw)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for i in range(n):
        po.render_camera(tree, cams[i % len(cams)], stop_T=STOP_T, out=img, aux_out=aux, **kw)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / n


def basis_leg(po, scenes, scene, cams, frames=50):
    """Colour-basis sweep (App. A basis ablation): the depth-9 geometry with
    SH-9, SH-16, SH-25 and SG-25 leaves (fresh N(0, 0.5^2) coefficients,
    lognormal densities as the main workload; SG lobes seeded), float32 and
    float16 leaves, 800x800 frames of the main poses."""
    res = {}
    for name, deg, sg in (("SH-9", 2, False), ("SH-16", 3, False), ("SH-25", 4, False), ("SG-25", 4, True)):
        sig, sh = scenes.leaf_values(len(scene["cells"]), deg, 1)
        sd = dict(scene, sh_degree=deg, sigma=sig, sh=sh)
        if sg:
            sd["lobes"] = scenes.sg_lobes((deg + 1) ** 2, 17)
        row = {}
        for dt in ("f32", "f16"):
            tree = po.Tree.from_scene(sd, dtype=dt)
            ms = _time_frames(po, tree, cams, frames)
            row[dt] = {"fps": round(1e3 / ms, 1), "leaf_bytes": (4 if dt == "f32" else 2) * (1 + 3 * tree.K),
                       "tree_mb": round(tree.nbytes() / 1e6, 1)}
            del tree
        res[name] = row
        log(f"basis {name}: {row}")
    return {"workload": "depth-9 blob band geometry, 800x800, %d frames per variant" % frames, "by_basis": res,
            "paper_context": {"fps": {"SH-9": 262, "SH-16": 168, "SH-25": 128, "SG-25": 151},
                              "hardware": "Tesla V100", "workload": "NeRF-synthetic real scenes"}}


def codebook_leg(po, scene, cams, frames=50, M=65536):
    """Codebook leaves (App. B.2) on the main workload: median-cut codebooks of
    2^16 float16 colours per basis function built on the host, 16-bit
    positions per leaf, float16 densities; render FPS, and the colour error
    of the compressed tree against the float32 tree's render of the same
    poses (quantisation error)."""
    import numpy as np
    import torch

    t0 = time.perf_counter()
    tree = po.Tree.from_cells_codebook(scene["depth"], scene["sh_degree"], scene["cells"], scene["sigma"],
                                       scene["sh"], M, scene["center"], scene["half"])
    t_build = time.perf_counter() - t0
    ms = _time_frames(po, tree, cams, frames)
    ref = po.Tree.from_scene(scene, dtype="f32")
    err_max, se, n = 0.0, 0.0, 0
    for c in cams[:4]:
        a = po.render_camera(ref, c, stop_T=STOP_T)
        b = po.render_camera(tree, c, stop_T=STOP_T)
        e = (a - b).abs()
        err_max = max(err_max, float(e.max()))
        se += float((e * e).sum())
        n += e.numel()
    mse = se / n
    rec = 2 + 2 * tree.K
    out = {"workload": "depth-9 blob band, SH-16, %d-entry float16 codebook per basis function" % M,
           "fps": round(1e3 / ms, 1), "build_s": round(t_build, 1),
           "leaf_bytes": rec, "leaf_bytes_f16": 2 * (1 + 3 * tree.K), "leaf_bytes_f32": 4 * (1 + 3 * tree.K),
           "codebook_mb": round(tree.codebook.numel() * 2 / 1e6, 1), "tree_mb": round(tree.nbytes() / 1e6, 1),
           "err_vs_f32_max": round(err_max, 5), "psnr_vs_f32": round(float(10 * np.log10(1.0 / max(mse, 1e-30))), 2)}
    del tree, ref
    torch.cuda.empty_cache()
    return out


def view_leg(po, tree, cams, frames=50):
    """Viewer outputs (Sec. 5.5) on the main workload: cost of the depth and
    alpha maps (aux output), of an SH subset and of a slicing plane relative
    to the plain render."""
    base = _time_frames(po, tree, cams, frames)
    depth = _time_frames(po, tree, cams, frames, aux=True)
    sub = _time_frames(po, tree, cams, frames, sh_off=0b1111111110000)
    cut = _time_frames(po, tree, cams, frames, clip=(0.3, -0.5, 0.8, 0.05))
    return {"fps_plain": round(1e3 / base, 1), "fps_depth_alpha": round(1e3 / depth, 1),
            "fps_sh_subset": round(1e3 / sub, 1), "fps_slicing_plane": round(1e3 / cut, 1)}


def filter_leg(po, tree, cams, tau=0.01):
    """Visibility filter (Sec. 4.2 "Filtering") on the main tree: alpha renders
    of the 800x800 poses raise each leaf's largest ray weight (atomic max);
    then the leaves below tau are pruned and the tree rebuilt on the host.
    Algorithmic bytes: per sample the density and the weight's read and
    write (12 B float32)."""
    import torch

    w = torch.zeros(tree.n_leaves, dtype=torch.float32, device="cuda")
    po.visibility.leaf_weights(tree, cams[:3], stop_T=STOP_T, weight=w)
    w.zero_()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    po.visibility.leaf_weights(tree, cams, stop_T=STOP_T, weight=w)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / len(cams)
    # samples per view from the render's aux pass (the filter walks the same segments)
    aux = torch.empty((H, W, po.AUX_WIDTH), dtype=torch.float32, device="cuda")
    n_samples = 0.0
    for c in cams[:20]:
        po.render_camera(tree, c, stop_T=STOP_T, aux=True, aux_out=aux)
        n_samples += float(aux[..., po.AUX_SAMPLES].double().sum())
    n_samples /= 20
    t0 = time.perf_counter()
    pruned, kept = po.visibility.prune(tree, w, tau)
    t_prune = time.perf_counter() - t0
    gbps = 12.0 * n_samples / (ms * 1e-3) / 1e9
    return {"views": len(cams), "ms_per_view": round(ms, 4), "mrays_per_s": round(W * H / (ms * 1e3), 1),
            "msamples_per_s": round(n_samples / (ms * 1e3), 1),
            "roofline": {"bound": "hbm", "achieved": round(gbps, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                         "frac": round(gbps / HBM_PEAK_GBPS, 4), "alg_bytes_per_sample": 12},
            "tau_w": tau, "leaves_kept": int(len(kept)), "leaves": int(tree.n_leaves),
            "prune_rebuild_s": round(t_prune, 2)}


def calib_copy(mib: int):
    """One plain device-to-device copy of `mib` MiB, for scaling the HBM
    traffic counters (it reads and writes exactly that many bytes)."""
    import torch

    a = torch.empty(mib << 20, dtype=torch.uint8, device="cuda")
    a.fill_(1)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    del a, b
    torch.cuda.empty_cache()


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-fp16", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-train", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=2000, help="requests per arrival rate")
    ap.add_argument("--no-extra", action="store_true", help="skip the viewer, filter and basis-sweep legs")
    ap.add_argument("--profile", action="store_true",
                    help="time the float32 renders only (no sample-count pass, fp16 or CPU legs); no JSON line")
    ap.add_argument("--train-only", action="store_true",
                    help="run the differentiation leg alone and print its JSON (for profiling)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="run one plain copy of this many MiB first (HBM counter calibration)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only (a render needs no communication between GPUs; several GPUs "
              "would each render their own frames or requests); rerun with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2103_14024_amd as po
    from paper_2103_14024_amd import scenes

    torch.cuda.set_device(0)
    if args.calib_copy_mib:
        calib_copy(args.calib_copy_mib)
    if args.train_only:
        # no dataset PSNR passes: the profile then holds the training steps
        print(json.dumps(train_leg(po, scenes, steps=args.steps, warmup=args.warmup, fit_steps=0, psnr=False)),
              flush=True)
        return
    t0 = time.perf_counter()
    scene = scenes.scene_blobs()
    log(f"scene: {len(scene['cells'])} leaves in {time.perf_counter() - t0:.1f} s")
    poses = scenes.hemisphere_poses(N_POSES, 4.0, 2)
    fx, fy, cx, cy = scenes.intrinsics(W, H, 40.0)
    cams = [po.Camera(p, W, H, fx, fy, cx, cy) for p in poses]
    stream = torch.cuda.current_stream()

    tree32 = po.Tree.from_scene(scene, dtype="f32")
    torch.cuda.synchronize()
    log(f"fp32 tree: {tree32.n_nodes} nodes, {tree32.nbytes() / 1e6:.0f} MB")
    if args.profile:
        r = measure(po, tree32, cams, args.steps, args.warmup, stream, aux_pass=False)
        log(f"profile run: {r['fps']:.1f} FPS, {r['ms_per_step']:.3f} ms per frame")
        return
    r32 = measure(po, tree32, cams, args.steps, args.warmup, stream)
    log(f"fp32: {r32['fps']:.1f} FPS, {r32['msamples_per_s']:.0f} Msamples/s, "
        f"{r32['samples_per_ray']:.2f} samples/ray, {r32['steps_per_ray']:.1f} steps/ray, "
        f"{r32['node_loads_per_ray']:.1f} child-entry reads/ray, lane efficiency {r32['lane_efficiency']:.3f}")
    frames32 = {} if args.no_cpu_baseline else gpu_frames(po, tree32, cams, ERR_POSES)
    one32 = measure_one_pass(po, tree32, cams, args.steps, args.warmup, stream)
    log(f"fp32 one pass: {one32['fps']:.1f} FPS")
    e2e = None if args.no_extra else measure_end_to_end(po, tree32, cams, args.steps, args.warmup, stream)
    if e2e:
        log(f"fp32 with the image copied to the host: {e2e}")
    tb = counter_traffic("f32")
    traffic_gbps = None if tb is None else round(tb / (r32["ms_per_step"] * 1e-3) / 1e9, 1)
    out = {
        "metric": METRIC, "value": round(r32["fps"], 2), "unit": "FPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(r32["ms_per_step"], 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "plenoctree-render depth-9 blob band, SH degree 3, 800x800, 200 hemisphere poses",
                   "leaves": int(len(scene["cells"])), "nodes": int(tree32.n_nodes), "depth": 9, "sh_degree": 3,
                   "width": W, "height": H, "poses": N_POSES, "poses_timed": r32["poses_timed"],
                   "stop_T": STOP_T, "leaf_dtype": "f32"},
        "msamples_per_s": round(r32["msamples_per_s"], 1), "mrays_per_s": round(r32["mrays_per_s"], 1),
        "samples_per_ray": round(r32["samples_per_ray"], 3), "steps_per_ray": round(r32["steps_per_ray"], 2),
        "child_entry_reads_per_ray": round(r32["node_loads_per_ray"], 2),
        "lane_efficiency": round(r32["lane_efficiency"], 4),
        "one_pass": one32,
        "end_to_end_with_d2h": e2e,
        "roofline": {"bound": "hbm", "achieved": round(r32["alg_gbps"], 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": round(r32["alg_gbps"] / HBM_PEAK_GBPS, 4), "traffic": traffic_gbps,
                     "kernel": "render pass <float,16,16,48,SH>: k_zero_i32, k_render_camera_split, "
                               "k_render_chunks, k_render_subchunks, k_render_join",
                     "alg_bytes_per_frame": int(r32["alg_bytes_per_launch"]),
                     "alg_bytes_per_frame_parts": {k: int(v) for k, v in r32["alg_bytes_split"].items()},
                     "hbm_bytes_per_frame": None if tb is None else int(tb)},
        "paper_context": {"fps": 167.68, "hardware": "Tesla V100", "workload": "NeRF-synthetic real scenes"},
    }
    if not args.no_extra:
        out["view"] = view_leg(po, tree32, cams)
        log(f"view: {out['view']}")
        out["filter"] = filter_leg(po, tree32, cams[:100])
        log(f"filter: {out['filter']}")
    del tree32
    torch.cuda.empty_cache()
    frames16 = {}
    if not args.no_fp16:
        tree16 = po.Tree.from_scene(scene, dtype="f16")
        r16 = measure(po, tree16, cams, args.steps, args.warmup, stream)
        log(f"fp16: {r16['fps']:.1f} FPS, {r16['msamples_per_s']:.0f} Msamples/s")
        one16 = measure_one_pass(po, tree16, cams, args.steps, args.warmup, stream)
        if not args.no_cpu_baseline:
            frames16 = gpu_frames(po, tree16, cams, ERR_POSES)
        t16 = counter_traffic("f16")
        out["fp16"] = {"fps": round(r16["fps"], 2), "ms_per_step": round(r16["ms_per_step"], 4),
                       "msamples_per_s": round(r16["msamples_per_s"], 1),
                       "alg_gbps": round(r16["alg_gbps"], 1), "alg_frac": round(r16["alg_gbps"] / HBM_PEAK_GBPS, 4),
                       "alg_bytes_per_frame": int(r16["alg_bytes_per_launch"]),
                       "hbm_gbps": None if t16 is None else round(t16 / (r16["ms_per_step"] * 1e-3) / 1e9, 1),
                       "speedup_vs_fp32": round(r16["fps"] / r32["fps"], 3), "one_pass": one16}
        del tree16
    if not args.no_extra:
        out["basis"] = basis_leg(po, scenes, scene, cams)
        out["codebook"] = codebook_leg(po, scene, cams)
        log(f"codebook: {out['codebook']}")
    if not args.no_train:
        log("differentiation: direct octree optimisation")
        out["train"] = train_leg(po, scenes)
        log(f"train: {out['train']['mrays_per_s']} Mrays/s, PSNR {out['train']['psnr_start']} -> "
            f"{out['train']['psnr_after']}")
    if not args.no_serve:
        out["serve"] = serve_leg(po, scenes, n_requests=args.serve_requests)
    if not args.no_cpu_baseline:
        log("cpu baseline (FP64 oracle) and the error of the GPU renders against it")
        out["cpu_baseline"], err = cpu_baseline(scene, poses, frames32, frames16)
        out["error_vs_fp64_oracle"] = {"poses": err["poses"], "pixels": err["pixels"],
                                       "f32": err["f32_vs_oracle"]}
        if "fp16" in out and "f16_vs_oracle_f32_values" in err:
            out["fp16"]["error_vs_fp64_oracle"] = {
                "poses": err["poses"], "pixels": err["pixels"],
                "vs_float32_values": err["f16_vs_oracle_f32_values"],
                "vs_float16_values": err["f16_vs_oracle_f16_values"]}
        log(f"error vs oracle: {err}")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
