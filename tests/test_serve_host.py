"""Host logic of the serving loop (admission by memory, FIFO batching,
overlap of batches across workers, rejection, error delivery), exercised on
the CPU with a stand-in batch renderer."""
import threading
import time

import numpy as np
import pytest

from paper_2504_12811_amd import scenes as S
from paper_2504_12811_amd.serve import AdmissionError, Server, estimate_bytes, random_request


class FakeRender:
    def __init__(self, delay=0.02):
        self.delay = delay
        self.calls = []  # (worker, t0, t1, n_views)
        self.lock = threading.Lock()

    def __call__(self, wid, cams):
        t0 = time.perf_counter()
        time.sleep(self.delay)
        t1 = time.perf_counter()
        with self.lock:
            self.calls.append((wid, t0, t1, len(cams)))
        # an "image" that identifies its camera
        return [np.full((1,), c.width * 10000 + c.height, np.int64) for c in cams], 100


def cam(w, h):
    return S.pinhole((0.0, 0.0, -5.0), w, h, 60.0)


def test_results_match_their_requests_and_batches_respect_the_limit():
    fr = FakeRender()
    with Server(fr, n_gaussians=1000, mem_cap=1 << 40, max_batch=4, n_workers=2) as srv:
        sizes = [(16 + k, 8 + k) for k in range(20)]
        futs = [srv.submit([cam(w, h)]) for (w, h) in sizes]
        res = [f.result(timeout=10) for f in futs]
    for (w, h), r in zip(sizes, res):
        assert int(r.images[0][0]) == w * 10000 + h
        assert r.latency >= 0
    assert max(srv.batches) <= 4 and sum(srv.batches) == 20


def test_memory_admission_bounds_in_flight_bytes():
    """Each worker renders into its share of the cap: a batch holds only as
    many requests as fit that share, and the bytes in flight never exceed
    the cap."""
    fr = FakeRender(0.01)
    one = estimate_bytes(1000, [cam(64, 64)])
    cap = int(2 * 2.5 * one)
    with Server(fr, n_gaussians=1000, mem_cap=cap, max_batch=8, n_workers=2) as srv:
        assert srv.worker_bytes == cap // 2
        futs = [srv.submit([cam(64, 64)]) for _ in range(12)]
        for f in futs:
            f.result(timeout=10)
        assert srv.peak_mem <= cap
        assert max(srv.batches) <= 2


def test_request_above_the_cap_is_rejected():
    fr = FakeRender()
    with Server(fr, n_gaussians=10_000_000, mem_cap=1 << 20, max_batch=4) as srv:
        f = srv.submit([cam(1920, 1080)])
        with pytest.raises(AdmissionError):
            f.result(timeout=5)


def test_request_above_a_workers_share_is_rejected():
    """A request whose records alone (no pair buffer) exceed one worker's
    share of the cap can never be rendered (a batch renders in one worker's
    workspace)."""
    fr = FakeRender()
    fixed = estimate_bytes(1000, [cam(64, 64)], 0.0)
    with Server(fr, n_gaussians=1000, mem_cap=int(1.5 * fixed), max_batch=4, n_workers=2) as srv:
        f = srv.submit([cam(64, 64)])
        with pytest.raises(AdmissionError):
            f.result(timeout=5)
    assert fr.calls == []


def test_request_whose_pair_estimate_exceeds_the_share_goes_alone():
    """The pair estimate is conservative: a request above the share whose
    records fit is rendered, in a batch of its own."""
    fr = FakeRender(0.01)
    one = estimate_bytes(1000, [cam(64, 64)])
    fixed = estimate_bytes(1000, [cam(64, 64)], 0.0)
    share = (fixed + one) // 2
    with Server(fr, n_gaussians=1000, mem_cap=2 * share, max_batch=4, n_workers=2) as srv:
        futs = [srv.submit([cam(64, 64)]) for _ in range(5)]
        for f in futs:
            f.result(timeout=10)
    assert srv.batches and max(srv.batches) == 1 and sum(srv.batches) == 5


def test_requests_arriving_during_a_batch_run_on_the_other_worker():
    fr = FakeRender(0.05)
    with Server(fr, n_gaussians=1000, mem_cap=1 << 40, max_batch=8, n_workers=2) as srv:
        f1 = srv.submit([cam(32, 32)])
        time.sleep(0.01)  # the first batch is now running
        f2 = [srv.submit([cam(40, 40)]) for _ in range(3)]
        f1.result(timeout=5)
        for f in f2:
            f.result(timeout=5)
    (w0, a0, b0, _), (w1, a1, b1, _) = sorted(fr.calls, key=lambda c: c[1])[:2]
    assert w0 != w1 and a1 < b0  # overlapped in time on different workers


def test_render_errors_reach_every_waiting_caller():
    def boom(wid, cams):
        raise RuntimeError("device error")
    with Server(boom, n_gaussians=10, mem_cap=1 << 40, max_batch=4, n_workers=1) as srv:
        futs = [srv.submit([cam(8, 8)]) for _ in range(3)]
        for f in futs:
            with pytest.raises(RuntimeError):
                f.result(timeout=5)


def test_random_requests_follow_the_workload():
    rng = np.random.default_rng(0)
    seen = set()
    for _ in range(300):
        cams = random_request(rng)
        c = cams[0]
        seen.add((c.width, c.height, len(cams)))
        fov = 2 * np.degrees(np.arctan(c.width / 2 / c.fx))
        assert 40 - 1e-9 <= fov <= 120 + 1e-9
        d = np.linalg.norm(c.position)
        assert 10 * np.sqrt(3) * 0.99 <= d <= 32 * 10 * np.sqrt(3) * 1.01
    assert (2160, 1200, 2) in seen and (256, 256, 1) in seen and len(seen) == 5
