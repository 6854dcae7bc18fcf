"""Serving: a resident scene, continuous batching of render requests.

Requests (one or two views each: a pinhole camera per view) enter a FIFO
queue.  Each worker owns a library context, a HIP stream and a workspace of
its share of the memory cap, allocated when the server starts, so nothing is
allocated on the request path and the workspaces never exceed the cap.  A
worker that becomes free takes, from the head of the queue, as many requests
as fit both the batch limit and its share of the cap (estimated device
memory of the batch), renders them with one batched launch sequence on its
stream into its workspace, and completes their futures.
Requests that arrive while batches are on the GPU are admitted as soon as a
worker and memory free up; with two or more workers, batches overlap on the
device.  Every view in a batch is bit-identical to rendering it alone (the
batched kernels run the same per-view arithmetic).

The admission and batching logic is plain Python and takes the batch render
function as a parameter, so it can be exercised without a GPU.
"""
from __future__ import annotations

import collections
import math
import threading
import time
from concurrent.futures import Future
from dataclasses import dataclass, field
from typing import Callable, List, Optional, Sequence

import numpy as np


class AdmissionError(RuntimeError):
    """The request can never fit under the memory cap."""


@dataclass
class Request:
    cams: list                    # one camera per view (two for a stereo request)
    t_arrival: float = 0.0
    future: Future = field(default_factory=Future)
    est_bytes: int = 0


@dataclass
class Result:
    images: list                  # [rgb [3,H,W]] per view (device tensors)
    t_arrival: float
    t_done: float
    batch_size: int               # requests in the batch this one was rendered with

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrival


def estimate_bytes(n_gaussians: int, cams, pairs_per_pixel: float = 2.0) -> int:
    """Device memory of one request: the per-(Gaussian, view) records and
    scratch (~420 B), the pair buffers (~51 B per pair incl. sort and emitter scratch,
    plus ~33 B per pair of long-list masks), per-pixel state and the output
    images."""
    pix = sum(int(c.width) * int(c.height) for c in cams)
    per_item = 4 + 16 + 16 + 4 + 128 + 128 + 4 + 8 + 4 + 96
    pairs = pairs_per_pixel * pix + 4096
    return int(n_gaussians * len(cams) * per_item + pairs * 84 + pix * (4 + 16 + 4) + (1 << 20))


class Server:
    """Continuous-batching render server (see module docstring).

    render_batch(worker_id, cams) -> (list of rgb per view, pairs) renders one
    batch on the worker's own stream and returns when it is done.
    """

    def __init__(self, render_batch: Callable, n_gaussians: int, mem_cap: int = 16 << 30, max_batch: int = 8,
                 n_workers: int = 2, pairs_per_pixel: float = 2.0):
        self._render_batch = render_batch
        self.n = n_gaussians
        self.mem_cap = int(mem_cap)
        self.max_batch = int(max_batch)
        self.n_workers = int(n_workers)
        # each worker renders into a workspace of its share of the cap
        self.worker_bytes = self.mem_cap // self.n_workers
        self.pairs_per_pixel = pairs_per_pixel
        self._q: collections.deque = collections.deque()
        self._cv = threading.Condition()
        self._mem_in_use = 0
        self._stop = False
        self.batches: List[int] = []   # sizes of the batches launched
        self.peak_mem = 0
        self._threads = [threading.Thread(target=self._worker, args=(w,), daemon=True) for w in range(n_workers)]
        for t in self._threads:
            t.start()

    # ------------------------------------------------------------------
    def submit(self, cams, t_arrival: Optional[float] = None) -> Future:
        req = Request(list(cams), time.perf_counter() if t_arrival is None else t_arrival)
        req.est_bytes = estimate_bytes(self.n, req.cams, self.pairs_per_pixel)
        fixed = estimate_bytes(self.n, req.cams, 0.0)  # without the pair buffers
        if fixed > self.worker_bytes:
            req.future.set_exception(AdmissionError(
                f"request needs ~{fixed >> 20} MiB before any pair, above a worker's {self.worker_bytes >> 20} MiB "
                f"share of the {self.mem_cap >> 20} MiB cap"))
            return req.future
        with self._cv:
            self._q.append(req)
            self._cv.notify()
        return req.future

    def close(self):
        with self._cv:
            self._stop = True
            self._cv.notify_all()
        for t in self._threads:
            t.join()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # ------------------------------------------------------------------
    def _take_batch(self) -> List[Request]:
        """Called with the lock held: FIFO requests that fit the batch limit
        and a worker's share of the cap.  A request whose estimate alone
        exceeds the share (the pair estimate is conservative) goes alone; its
        worker renders it with the pair buffer that fits, and reports it
        rejected if its pairs do not."""
        batch, need = [], 0
        while self._q and len(batch) < self.max_batch:
            r = self._q[0]
            if need + r.est_bytes > self.worker_bytes and batch:
                break
            batch.append(self._q.popleft())
            need += r.est_bytes
            if need > self.worker_bytes:
                break
        if batch:
            need = min(need, self.worker_bytes)
            self._mem_in_use += need
            self.peak_mem = max(self.peak_mem, self._mem_in_use)
            self.batches.append(len(batch))
        return batch

    def _worker(self, wid: int):
        while True:
            with self._cv:
                batch = self._take_batch()
                while not batch:
                    if self._stop and not self._q:
                        return
                    self._cv.wait()
                    batch = self._take_batch()
            cams = [c for r in batch for c in r.cams]
            try:
                images, pairs = self._render_batch(wid, cams)
                t_done = time.perf_counter()
                k = 0
                for r in batch:
                    imgs = images[k: k + len(r.cams)]
                    k += len(r.cams)
                    r.future.set_result(Result(imgs, r.t_arrival, t_done, len(batch)))
                pix = sum(int(c.width) * int(c.height) for c in cams)
                if pairs is not None and pix > 0:
                    # learn the pair density for the admission estimate
                    self.pairs_per_pixel = max(self.pairs_per_pixel * 0.98, 1.25 * pairs / pix, 0.5)
            except Exception as e:  # noqa: BLE001 - delivered to every waiting caller
                for r in batch:
                    if not r.future.done():
                        r.future.set_exception(e)
            finally:
                with self._cv:
                    self._mem_in_use -= min(sum(r.est_bytes for r in batch), self.worker_bytes)
                    self._cv.notify_all()


def gpu_render_batch(scene, settings, n_workers: int, device: int = 0, worker_bytes: int = 8 << 30):
    """Batch render functions for `Server`: one rasteriser (library
    context), one HIP stream and one workspace of `worker_bytes` per worker,
    allocated here.  A batch renders into its worker's workspace with the
    largest pair buffer that fits; if its pairs overflow that buffer it is
    rendered in two halves (a single view that cannot fit raises)."""
    import torch
    from . import _lib as L
    from .render import Rasterizer, Workspace

    rasters = [Rasterizer(device) for _ in range(n_workers)]
    streams = [torch.cuda.Stream(device=device) for _ in range(n_workers)]
    spaces = [Workspace(torch.device("cuda", device), int(worker_bytes), 0) for _ in range(n_workers)]

    def render(wid, cams):
        ras, ws = rasters[wid], spaces[wid]
        mp = ras.batch_pair_capacity(scene, cams, settings, ws.nbytes)
        try:
            if mp <= 0:
                raise L.AAAError(L.AAA_ERR_WORKSPACE, "batch does not fit the worker's workspace")
            rgbs, _, st = ras.render_batch(scene, cams, settings, ws=ws, max_pairs=mp)
            return rgbs, int(st.pairs)
        except L.AAAError as e:
            if e.code not in (L.AAA_ERR_PAIR_OVERFLOW, L.AAA_ERR_WORKSPACE):
                raise
            if len(cams) == 1:
                raise AdmissionError(f"view does not fit the worker's {ws.nbytes >> 20} MiB workspace: {e}") from e
        h = len(cams) // 2
        a, pa = render(wid, cams[:h])
        b, pb = render(wid, cams[h:])
        return a + b, pa + pb

    def fn(wid: int, cams):
        with torch.cuda.stream(streams[wid]):
            rgbs, pairs = render(wid, cams)
            streams[wid].synchronize()
        return rgbs, pairs

    fn.worker_bytes = int(worker_bytes)
    return fn


# ----------------------------------------------------------------------
# synthetic request stream (the serving workload)

RESOLUTIONS = [(256, 256), (640, 480), (1280, 720), (1920, 1080), (2160, 1200)]  # the last: per eye, two views
EYE_SEPARATION = 0.063


def random_request(rng: np.random.Generator, scene_radius: float = 10.0 * math.sqrt(3.0)):
    """A pose on a random direction at distance U[1, 32] scene radii looking at
    the origin, resolution uniform over RESOLUTIONS, horizontal FoV
    U[40, 120] deg; the stereo resolution gives two views 0.063 apart."""
    from .scenes import Camera, look_at, pinhole
    d = rng.normal(size=3)
    d /= np.linalg.norm(d)
    dist = rng.uniform(1.0, 32.0) * scene_radius
    w, h = RESOLUTIONS[int(rng.integers(0, len(RESOLUTIONS)))]
    fov = rng.uniform(40.0, 120.0)
    pos = d * dist
    if (w, h) == (2160, 1200):
        c = pinhole(pos, w, h, fov)
        right = c.viewmat[0, :3]
        return [pinhole(pos - 0.5 * EYE_SEPARATION * right, w, h, fov),
                pinhole(pos + 0.5 * EYE_SEPARATION * right, w, h, fov)]
    return [pinhole(pos, w, h, fov)]


def run_load(server: Server, rate: float, duration: float, seed: int = 7, max_requests: Optional[int] = None):
    """Open-loop Poisson arrivals at `rate` req/s for `duration` seconds;
    returns (latencies [s], frames completed, wall time, rejected)."""
    rng = np.random.default_rng(seed)
    futs = []
    t0 = time.perf_counter()
    t_next = t0
    while True:
        t_next += rng.exponential(1.0 / rate)
        if t_next - t0 > duration or (max_requests and len(futs) >= max_requests):
            break
        delay = t_next - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        futs.append(server.submit(random_request(rng), t_arrival=t_next))
    lat, frames, rejected = [], 0, 0
    for f in futs:
        try:
            r = f.result()
        except AdmissionError:
            rejected += 1
            continue
        lat.append(r.latency)
        frames += len(r.images)
    wall = time.perf_counter() - t0
    return np.asarray(lat), frames, wall, rejected
