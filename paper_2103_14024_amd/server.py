"""Continuous-batching render server over several scenes resident in HBM.

Requests (scene, camera) arrive over time.  The loop admits arrived requests
while their output images fit an HBM budget and a slot cap.  A request of at
least `split_tiles` 16x16 tiles is rendered whole by one job, which the
library renders in pieces (long walks cut and walked in parallel); smaller
requests are cut into chunks of tiles, and chunks of several requests -- of
any scene and resolution -- are packed into batched launches
(po_render_batch, up to 16 jobs each), each ray of a chunk walked by one
lane (one pass).  Launches go round-robin to a few HIP
streams, so a large frame and the batches of small ones run on the device
together.  Requests that arrive while others are in flight join the next
launch.  A request is complete when the last launch holding one of its tiles
has finished; latency is measured from its arrival to that launch's
completion on the GPU clock (HIP events).

The rendering itself is the library's; this module is scheduling only.
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

from . import _lib as L
from .render import Camera, Job, render_batch

_ALIGN = 256


@dataclass
class Request:
    rid: int
    scene: int
    cam: Camera
    arrival: float                      # seconds since the start of the run
    # filled in by the server
    offset: int = -1
    tiles: int = 0
    next_tile: int = 0
    done_tiles: int = 0
    t_admit: float = float("nan")
    t_done: float = float("nan")
    image: object = None                # host copy when kept

    @property
    def nbytes(self) -> int:
        return self.cam.width * self.cam.height * 3 * 4


class Arena:
    """First-fit allocator over one preallocated device buffer (the HBM
    budget for output images)."""

    def __init__(self, nbytes: int, device="cuda"):
        import torch

        self.size = int(nbytes)
        self.buf = torch.empty(self.size, dtype=torch.uint8, device=device)
        self.free = [(0, self.size)]    # sorted (offset, length)
        self.used = 0

    def alloc(self, n: int) -> int:
        n = (n + _ALIGN - 1) // _ALIGN * _ALIGN
        for i, (o, ln) in enumerate(self.free):
            if ln >= n:
                if ln == n:
                    self.free.pop(i)
                else:
                    self.free[i] = (o + n, ln - n)
                self.used += n
                return o
        return -1

    def release(self, o: int, n: int) -> None:
        n = (n + _ALIGN - 1) // _ALIGN * _ALIGN
        self.used -= n
        self.free.append((o, n))
        self.free.sort()
        merged = []
        for a, ln in self.free:
            if merged and merged[-1][0] + merged[-1][1] == a:
                merged[-1] = (merged[-1][0], merged[-1][1] + ln)
            else:
                merged.append((a, ln))
        self.free = merged

    def view(self, req: Request):
        return self.buf[req.offset:req.offset + req.nbytes].view(dtype=__import__("torch").float32).view(
            req.cam.height, req.cam.width, 3)


@dataclass
class Stats:
    latencies_ms: list = field(default_factory=list)
    wall_s: float = 0.0
    pixels: int = 0
    launches: int = 0
    jobs: int = 0
    max_jobs: int = 0                   # most jobs in one launch
    whole: int = 0                      # requests rendered whole, in pieces
    max_active: int = 0
    max_bytes: int = 0

    def summary(self) -> dict:
        lat = np.asarray(self.latencies_ms)
        return {"requests": int(len(lat)), "p50_ms": round(float(np.percentile(lat, 50)), 3),
                "p99_ms": round(float(np.percentile(lat, 99)), 3), "mean_ms": round(float(lat.mean()), 3),
                "throughput_req_s": round(len(lat) / self.wall_s, 2),
                "mrays_per_s": round(self.pixels / self.wall_s / 1e6, 2), "launches": self.launches,
                "jobs_per_launch": round(self.jobs / max(1, self.launches), 2), "max_jobs_per_launch": self.max_jobs,
                "rendered_whole": self.whole, "max_active": self.max_active,
                "max_output_mb": round(self.max_bytes / 1e6, 1)}


class Server:
    """Continuous-batching scheduler.

    trees: resident scenes; budget_bytes: HBM for output images; max_active:
    admitted-request slots; chunk_tiles: least tiles of one request per
    launch; launch_tiles: tiles per launch; streams: HIP streams used round-robin;
    max_inflight: launches queued on the GPU at once; split_tiles: requests of
    at least this many tiles are rendered whole, in pieces (None: never)."""

    def __init__(self, trees, budget_bytes=512 << 20, max_active=64, chunk_tiles=256, launch_tiles=2048,
                 streams=3, max_inflight=4, stop_T=1e-4, bg=(1.0, 1.0, 1.0), device="cuda", split_tiles=1024):
        import torch

        self.trees = list(trees)
        self.arena = Arena(budget_bytes, device)
        self.max_active, self.chunk_tiles, self.launch_tiles = max_active, chunk_tiles, launch_tiles
        self.streams = [torch.cuda.Stream(device=device) for _ in range(streams)]
        self.max_inflight = max_inflight
        self.stop_T, self.bg = stop_T, tuple(bg)
        self.split_tiles = split_tiles if split_tiles is not None else 1 << 30

    def run(self, requests, keep_images=False, on_complete=None) -> Stats:
        """Serves `requests` (sorted by arrival) in real time; returns Stats."""
        import torch

        for r in requests:
            if r.nbytes > self.arena.size:
                raise ValueError(f"request {r.rid} needs {r.nbytes} bytes, more than the budget")
        st = Stats()
        pending = deque(requests)
        waiting = deque()
        active = []
        inflight = []                       # (event, [(req, n_tiles)])
        ref = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        ref.record()
        ref.synchronize()
        t0 = time.perf_counter()
        k_stream = 0
        while pending or waiting or active or inflight:
            now = time.perf_counter() - t0
            while pending and pending[0].arrival <= now:
                waiting.append(pending.popleft())
            # retire finished launches (any order across streams)
            still = []
            for ev, parts in inflight:
                if ev.query():
                    t_gpu = ref.elapsed_time(ev) * 1e-3
                    for req, n in parts:
                        req.done_tiles += n
                        if req.done_tiles == req.tiles:
                            req.t_done = t_gpu
                            st.latencies_ms.append((req.t_done - req.arrival) * 1e3)
                            st.pixels += req.cam.width * req.cam.height
                            if keep_images:
                                req.image = self.arena.view(req).cpu().numpy()
                            if on_complete is not None:
                                on_complete(req, self.arena.view(req))
                            self.arena.release(req.offset, req.nbytes)
                            active.remove(req)
                else:
                    still.append((ev, parts))
            inflight = still
            # admission by slots and output memory
            while waiting and len(active) < self.max_active:
                req = waiting[0]
                off = self.arena.alloc(req.nbytes)
                if off < 0:
                    break
                waiting.popleft()
                req.offset, req.tiles, req.next_tile, req.t_admit = off, req.cam.n_tiles, 0, now
                active.append(req)
            st.max_active = max(st.max_active, len(active))
            st.max_bytes = max(st.max_bytes, self.arena.used)
            # pack one launch: oldest requests first; the launch's tile budget is
            # shared among the requests with work left, but no request gets less
            # than chunk_tiles (so a lone request still fills the GPU)
            if len(inflight) < self.max_inflight:
                # the oldest large request not started yet: whole, in pieces
                big = next((r for r in active if r.next_tile == 0 and r.tiles >= self.split_tiles), None)
                if big is not None:
                    s = self.streams[k_stream % len(self.streams)]
                    k_stream += 1
                    render_batch([Job(self.trees[big.scene], big.cam, self.arena.view(big), 0, big.tiles, self.bg,
                                      self.stop_T)], stream=s)
                    big.next_tile = big.tiles
                    ev = torch.cuda.Event(enable_timing=True)
                    ev.record(s)
                    inflight.append((ev, [(big, big.tiles)]))
                    st.launches += 1
                    st.jobs += 1
                    st.whole += 1
                    st.max_jobs = max(st.max_jobs, 1)
                    continue
                jobs, parts, budget = [], [], self.launch_tiles
                n_open = sum(1 for r in active if r.next_tile < r.tiles)
                share = max(self.chunk_tiles, self.launch_tiles // max(1, n_open))
                for req in active:
                    if req.next_tile >= req.tiles or (req.next_tile == 0 and req.tiles >= self.split_tiles):
                        continue
                    n = min(share, req.tiles - req.next_tile, budget)
                    if n <= 0 or len(jobs) == L.PO_BATCH_MAX_JOBS:
                        break
                    # batched chunks walk each ray in one lane (one_pass), so a
                    # request's pixels do not depend on how it was cut or batched
                    jobs.append(Job(self.trees[req.scene], req.cam, self.arena.view(req), req.next_tile,
                                    req.next_tile + n, self.bg, self.stop_T, one_pass=True))
                    parts.append((req, n))
                    req.next_tile += n
                    budget -= n
                if jobs:
                    s = self.streams[k_stream % len(self.streams)]
                    k_stream += 1
                    render_batch(jobs, stream=s)
                    ev = torch.cuda.Event(enable_timing=True)
                    ev.record(s)
                    inflight.append((ev, parts))
                    st.launches += 1
                    st.jobs += len(jobs)
                    st.max_jobs = max(st.max_jobs, len(jobs))
                    continue
            if not inflight and not active and not waiting and pending:
                dt = pending[0].arrival - (time.perf_counter() - t0)
                if dt > 2e-4:
                    time.sleep(dt - 1e-4)
        st.wall_s = time.perf_counter() - t0
        return st


RESOLUTIONS = [(256, 256), (512, 512), (800, 800), (1280, 720), (1920, 1080)]


def poisson_requests(n, rate, n_scenes, seed=0, fov_x_deg=40.0, radius=4.0):
    """n requests with exponential inter-arrival times (Poisson process of
    `rate` per second), a uniform scene, a uniform resolution from
    RESOLUTIONS and a random upper-hemisphere pose each."""
    from .scenes import hemisphere_poses, intrinsics

    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, n)
    arr = np.cumsum(gaps)
    sc = rng.integers(0, n_scenes, n)
    res = rng.integers(0, len(RESOLUTIONS), n)
    poses = hemisphere_poses(n, radius, seed + 1)
    out = []
    for i in range(n):
        W, H = RESOLUTIONS[res[i]]
        fx, fy, cx, cy = intrinsics(W, H, fov_x_deg)
        out.append(Request(i, int(sc[i]), Camera(poses[i], W, H, fx, fy, cx, cy), float(arr[i])))
    return out
