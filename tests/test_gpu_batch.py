"""Batches of views on the GPU: every view of a batch is bit-identical to
its single-view render; the multi-view backward equals the oracle's summed
gradient; the serving loop returns, for each request in a concurrent mix,
exactly the image of that request rendered alone."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2504_12811_amd import scenes as S

pytestmark = pytest.mark.gpu

GROUPS = ["means", "log_scales", "quats", "opacity_logits", "sh"]


@pytest.fixture(scope="module")
def ras():
    from paper_2504_12811_amd.render import Rasterizer
    return Rasterizer(0)


def test_batch_views_equal_single_renders(ras):
    from paper_2504_12811_amd.render import DeviceScene
    scene, poses = S.cluster_scene(50_000, seed=1002, n_rig=8)
    ds = DeviceScene.from_host(scene, "cuda:0")
    cams = [S.pinhole(poses[0], 320, 200, 60.0), S.pinhole(poses[1], 97, 131, 100.0, bg=(0.2, 0.3, 0.4)),
            S.pinhole(poses[2] * 3.0, 640, 480, 45.0), S.pinhole(poses[3], 16, 16, 60.0)]
    st = S.Settings()
    rgbs, Ts, stats = ras.render_batch(ds, cams, st)
    total = 0
    for c, rgb, T in zip(cams, rgbs, Ts):
        r1, T1, s1 = ras.render(ds, c, st)
        total += s1.pairs
        assert torch.equal(rgb, r1) and torch.equal(T, T1)
    assert stats.pairs == total


def test_batch_backward_equals_oracle_sum(ras):
    from paper_2504_12811_amd.render import DeviceScene
    scene, cam0 = S.small_scene(n=1500, seed=21, sh_degree=2)
    cams = [cam0, S.pinhole(cam0.position * 1.3, 96, 80, 70.0), S.pinhole(-cam0.position, 64, 64, 50.0)]
    st = S.Settings()
    rng = np.random.default_rng(3)
    gs, ref = [], None
    for c in cams:
        g = rng.normal(size=(3, c.height, c.width))
        base = O.render_backward(scene, c, st, g)
        g = g * (base.flags == 0)
        r = O.render_backward(scene, c, st, g)
        gs.append(g)
        ref = r if ref is None else type(r)(*[getattr(ref, f) + getattr(r, f) if f in GROUPS else getattr(r, f)
                                               for f in r.__dataclass_fields__])
    ds = DeviceScene.from_host(scene, "cuda:0")
    rgbs, Ts, _ = ras.render_batch(ds, cams, st, fresh_ws=True)
    grads = ras.backward_batch(ds, cams, st, ras.last_ws, rgbs,
                               [torch.from_numpy(g.astype(np.float32)).cuda() for g in gs])
    for k in GROUPS:
        a = grads[k].cpu().numpy().astype(np.float64)
        b = getattr(ref, k)
        print(k, np.abs(b).max(), np.abs(a - b).max(), flush=True)
        assert np.abs(a - b).max() <= 1e-4 * np.abs(b).max() + 1e-7, k


def test_server_results_equal_solo_renders(ras):
    from paper_2504_12811_amd.render import DeviceScene
    from paper_2504_12811_amd.serve import Server, gpu_render_batch, random_request
    scene, _ = S.cluster_scene(100_000, seed=1002, n_rig=4)
    ds = DeviceScene.from_host(scene, "cuda:0")
    st = S.Settings()
    rng = np.random.default_rng(11)
    # requests as drawn: mixed resolutions (stereo pairs included), fields of
    # view and zoom distances
    reqs = [random_request(rng) for _ in range(12)]
    fov = lambda c: round(float(np.degrees(2 * np.arctan(c.width / 2 / c.fx))), 1)
    print("requests (views, W, H, fov):", [(len(r), r[0].width, r[0].height, fov(r[0])) for r in reqs], flush=True)
    fn = gpu_render_batch(ds, st, n_workers=2, worker_bytes=4 << 30)
    with Server(fn, n_gaussians=ds.n, mem_cap=8 << 30, max_batch=4, n_workers=2) as srv:
        futs = [srv.submit(r) for r in reqs]
        results = [f.result(timeout=120) for f in futs]
    print("batch sizes:", srv.batches, flush=True)
    assert max(srv.batches) > 1  # requests were batched
    for r, res in zip(reqs, results):
        for c, img in zip(r, res.images):
            solo, _, _ = ras.render(ds, c, st)
            assert torch.equal(img, solo)
