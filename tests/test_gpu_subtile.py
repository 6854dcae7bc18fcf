"""The middle level of the hierarchical sort (AAA_SUBTILE_SORT: one exactly
depth-ordered list per 8x8 sub-tile, keyed by the depth on the sub-tile-centre
line) against the oracle's sub-tile ordering, through the C ABI: images at
several window sizes (K = 0 is where the sub-tile order shows directly),
ragged images, the 1M benchmark scene on sampled tiles, and gradients."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2504_12811_amd import scenes as S

from test_gpu_backward import compare_grads
from test_gpu_forward import compare_image, dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ras():
    from paper_2504_12811_amd.render import Rasterizer
    assert torch.cuda.is_available()
    return Rasterizer(0)


@pytest.mark.parametrize("K", [0, 4, 16])
def test_subtile_image_small(ras, K):
    scene, cam = S.small_scene()
    compare_image(ras, scene, cam, S.Settings(ray_window=K, subtile_sort=True), label=f"sub-tile C1 K={K}")


def test_subtile_order_differs_from_tile_order(ras):
    """With the window off, the sub-tile level changes the image (the tile
    level alone blends by the tile-centre depth), and both match their
    oracle."""
    scene, cam = S.small_scene(n=3000, seed=42, sh_degree=3)
    a = compare_image(ras, scene, cam, S.Settings(ray_window=0), label="tile level K=0")[0]
    b = compare_image(ras, scene, cam, S.Settings(ray_window=0, subtile_sort=True), label="sub-tile level K=0")[0]
    assert float((a - b).abs().max()) > 1e-3


def test_subtile_ragged_cluster(ras):
    scene, poses = S.cluster_scene(30_000, seed=1002, n_rig=8)
    cam = S.pinhole(poses[0], 250, 170, 60.0)
    for K in (0, 16):
        compare_image(ras, scene, cam, S.Settings(ray_window=K, subtile_sort=True), label=f"sub-tile 30k K={K}")


def test_subtile_headline_sampled(ras):
    scene, cams = S.headline()
    cam = cams[0]
    tx, ty = cam.tiles
    sel = np.zeros(tx * ty, np.uint8)
    sel[np.random.default_rng(4).choice(tx * ty, 16, replace=False)] = 1
    compare_image(ras, scene, cam, S.Settings(subtile_sort=True), tile_sel=sel, label="sub-tile 1M 1080p")


def test_subtile_pair_count(ras):
    """Each kept (Gaussian, tile) pair becomes one pair per 8x8 sub-tile its
    screen box reaches: between one and four."""
    scene, cam = S.small_scene()
    ds = dev(scene)
    _, _, s0 = ras.render(ds, cam, S.Settings(), stats=True)
    _, _, s1 = ras.render(ds, cam, S.Settings(subtile_sort=True), stats=True)
    assert s0.pairs <= s1.pairs <= 4 * s0.pairs


@pytest.mark.parametrize("K", [0, 16])
def test_subtile_backward(ras, K):
    scene, cam = S.small_scene(n=2000, sh_degree=1)
    compare_grads(ras, scene, cam, S.Settings(ray_window=K, subtile_sort=True), seed=K, label=f"sub-tile C1 K={K}")
