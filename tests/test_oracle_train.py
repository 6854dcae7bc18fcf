"""Pins of the oracle's training-side functions on constructed cases whose
answer follows from the definition by hand: the training sampling frequency
(Sec. 3.2: the maximum of f / d over the training cameras, d the view-space
depth of the mean) and the Adam step's bias correction."""
import numpy as np

from oracle import oracle as O
from paper_2504_12811_amd import scenes as S


def _cam_at(pos, w=200, h=100, fov=60.0, target=(0.0, 0.0, 0.0)):
    return S.pinhole(np.asarray(pos, float), w, h, fov, target=target)


def test_on_axis_is_focal_over_distance():
    cam = _cam_at((0.0, 0.0, -4.0))
    v, fl = O.training_frequency(np.zeros((3, 1)), [cam])
    assert v[0] == cam.fx / 4.0 and fl[0] == 0


def test_depth_is_the_view_z_not_the_distance():
    # an off-axis mean in the plane z = 0 seen from (0, 0, -4): depth 4, distance 5
    cam = _cam_at((0.0, 0.0, -4.0), w=400, h=400, fov=120.0)
    v, _ = O.training_frequency(np.array([[3.0], [0.0], [0.0]]), [cam])
    np.testing.assert_allclose(v[0], cam.fx / 4.0, rtol=1e-15)


def test_maximum_over_cameras_that_see_the_mean():
    near = _cam_at((0.0, 0.0, -2.0))
    far = _cam_at((0.0, 0.0, -5.0), w=800, h=400)  # larger fx, still smaller fx/d
    v, _ = O.training_frequency(np.zeros((3, 1)), [far, near])
    np.testing.assert_allclose(v[0], max(near.fx / 2.0, far.fx / 5.0), rtol=1e-15)
    assert near.fx / 2.0 != far.fx / 5.0


def test_seeing_cameras_take_precedence():
    # the near camera looks away (mean in front of it but outside its image);
    # the far camera sees the mean: the far one defines the value even though
    # the near one has the larger f / d
    near = _cam_at((0.0, 0.0, -1.0), fov=30.0, target=(3.0, 0.0, -1.0 + 1.0))
    far = _cam_at((0.0, 0.0, -10.0))
    mu = np.zeros((3, 1))
    X = near.viewmat[:3, :3] @ mu[:, 0] + near.viewmat[:3, 3]
    assert X[2] > near.znear
    x = near.cx + near.fx * X[0] / X[2]
    assert not (0 <= x <= near.width)
    assert near.fx / X[2] > far.fx / 10.0
    v, _ = O.training_frequency(mu, [near, far])
    np.testing.assert_allclose(v[0], far.fx / 10.0, rtol=1e-15)


def test_fallback_to_cameras_in_front():
    # no camera sees the mean: the maximum over cameras with the mean in front
    a = _cam_at((0.0, 0.0, -2.0), fov=20.0, target=(5.0, 0.0, -2.0 + 1.0))
    b = _cam_at((0.0, 0.0, 3.0), fov=20.0, target=(-5.0, 0.0, 2.0))
    mu = np.zeros((3, 1))
    za = (a.viewmat[:3, :3] @ mu[:, 0] + a.viewmat[:3, 3])[2]
    zb = (b.viewmat[:3, :3] @ mu[:, 0] + b.viewmat[:3, 3])[2]
    assert za > 0 and zb > 0
    v, _ = O.training_frequency(mu, [a, b])
    np.testing.assert_allclose(v[0], max(a.fx / za, b.fx / zb), rtol=1e-15)


def test_behind_every_camera_is_unclamped():
    cams = [_cam_at((0.0, 0.0, -4.0), target=(0.0, 0.0, -8.0)), _cam_at((0.0, 3.0, 0.0), target=(0.0, 6.0, 0.0))]
    v, _ = O.training_frequency(np.zeros((3, 1)), cams)
    assert np.isinf(v[0]) and v[0] > 0


def test_near_plane_and_border_decisions_are_flagged():
    cam = _cam_at((0.0, 0.0, -4.0))
    # a mean exactly at the near plane depth, and one projecting onto the left border
    zn = cam.znear
    mu_near = np.array([[0.0], [0.0], [-4.0 + zn]])
    # x = cx + fx X / z = 0  ->  X = -cx z / fx at depth 4
    mu_border = np.array([[-cam.cx * 4.0 / cam.fx], [0.0], [0.0]])
    _, fl = O.training_frequency(np.concatenate([mu_near, mu_border], axis=1), [cam])
    assert fl.tolist() == [1, 1]


def test_no_cameras_gives_infinity():
    v, _ = O.training_frequency(np.zeros((3, 3)), [])
    assert np.all(np.isinf(v))


# ---------------------------------------------------------------------------
# Adam (optimiser of the multi-view training step): bias-correction pins


def test_adam_first_step_is_lr_times_sign():
    g = np.array([3.0, -0.5, 1e-3, -7.0])
    p, m, v = O.adam_step(np.zeros(4), g, np.zeros(4), np.zeros(4), 1, lr=0.01, eps=0.0)
    np.testing.assert_allclose(p, -0.01 * np.sign(g), rtol=1e-13)


def test_adam_constant_gradient_moves_lr_per_step():
    g = np.array([2.0, -4.0])
    p, m, v = np.zeros(2), np.zeros(2), np.zeros(2)
    for t in range(1, 30):
        p_new, m, v = O.adam_step(p, g, m, v, t, lr=0.05, eps=0.0)
        np.testing.assert_allclose(p_new - p, -0.05 * np.sign(g), rtol=1e-10)
        p = p_new


def test_adam_zero_gradient_keeps_parameters():
    p0 = np.array([1.0, -2.0])
    p, m, v = O.adam_step(p0, np.zeros(2), np.zeros(2), np.zeros(2), 1, lr=0.1, eps=1e-8)
    assert np.array_equal(p, p0)
