"""Multi-view training step on the GPU: the Adam kernel against the FP64
oracle step on the same gradients, and a few training steps lowering the
L1 loss of a 4-view batch."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2504_12811_amd import scenes as S

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,offset", [(1, 0), (7, 0), (1003, 1), (1_000_003, 0)])
def test_adam_kernel_matches_oracle(n, offset):
    from paper_2504_12811_amd import _lib as L
    rng = np.random.default_rng(n)
    lr = 1e-2
    p0 = rng.normal(size=n).astype(np.float32)
    buf = {k: torch.zeros(n + offset, dtype=torch.float32, device="cuda") for k in ("p", "g", "m", "v")}
    P, G, M, V = (buf[k][offset:] for k in ("p", "g", "m", "v"))  # offset 1: unaligned, scalar path
    P.copy_(torch.from_numpy(p0))
    pr, mr, vr = p0.astype(np.float64), np.zeros(n), np.zeros(n)
    for t in range(1, 4):
        g = (rng.normal(size=n) * 10.0 ** rng.uniform(-3, 1, size=n)).astype(np.float32)
        G.copy_(torch.from_numpy(g))
        L.check(L.lib().aaa_adam_step(P.data_ptr(), G.data_ptr(), M.data_ptr(), V.data_ptr(), n, t, lr, 0.9, 0.999,
                                      1e-15, torch.cuda.current_stream().cuda_stream))
        pr, mr, vr = O.adam_step(pr, g, mr, vr, t, lr, eps=1e-15)
    torch.cuda.synchronize()
    got = P.cpu().numpy().astype(np.float64)
    # float32 state: each update carries a relative error of a few ulps
    # (<= 4e-6 * lr with margin), the parameter is rounded to float32 after
    # every step (<= 6e-8 |p|, taken twice)
    err = np.abs(got - pr)
    bound = 3 * (4e-6 * lr + 1.2e-7 * np.abs(pr))
    print(f"n={n} max err {err.max():.3e}")
    assert np.all(err <= bound)


def test_adam_rejects_bad_arguments():
    from paper_2504_12811_amd import _lib as L
    x = torch.zeros(4, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    for args in [(4, 0, 1e-3, 0.9, 0.999, 1e-8), (4, 1, 1e-3, 1.0, 0.999, 1e-8), (4, 1, 1e-3, 0.9, 0.999, 0.0),
                 (-1, 1, 1e-3, 0.9, 0.999, 1e-8)]:
        assert L.lib().aaa_adam_step(x.data_ptr(), x.data_ptr(), x.data_ptr(), x.data_ptr(), *args, s) == \
            L.AAA_ERR_INVALID


def test_training_steps_lower_the_loss():
    from paper_2504_12811_amd.render import DeviceScene, Rasterizer
    from paper_2504_12811_amd.train import Adam, train_step
    ras = Rasterizer(0)
    scene, poses = S.cluster_scene(20_000, seed=1004, n_rig=4, rig_w=160, rig_h=90, rig_fov=70.0)
    cams = [S.pinhole(p, 160, 90, 70.0) for p in poses]
    st = S.Settings()
    # targets: renders of a perturbed copy of the scene
    tgt_scene = S.Scene(scene.means, scene.log_scales + 0.2, scene.quats, scene.opacity_logits + 0.5, scene.sh,
                        scene.v_train)
    tds = DeviceScene.from_host(tgt_scene, "cuda:0")
    targets = [ras.render(tds, c, st)[0].clone() for c in cams]
    ds = DeviceScene.from_host(scene, "cuda:0")
    opt = Adam(ds)
    losses = [train_step(ras, ds, cams, targets, st, opt) for _ in range(15)]
    print("losses", [round(l, 5) for l in losses])
    assert all(np.isfinite(losses))
    assert losses[-1] < 0.8 * losses[0]
