"""Checkpoints on the GPU: a tree written with Tree.save and bound again with
Tree.load renders bit for bit like the original (float32, float16,
spherical-Gaussian and codebook leaves, split and one-pass sizes), and a
Trainer resumed from its checkpoint continues the same fit (same step count,
same batch draws, same leaf values up to the order of the gradient atomics)."""
import sys

import numpy as np
import pytest

from paper_2103_14024_amd import scenes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def po():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2103_14024_amd as po

    po.reset_device_errors()
    return po


def _announce(msg):
    print(f"[gpu] {msg}", file=sys.stderr, flush=True)


@pytest.mark.parametrize("form", ["f32", "f16", "sg", "codebook"])
def test_tree_round_trip_renders_identically(po, tmp_path, form):
    import torch

    _announce(f"checkpoint round trip {form}")
    s = scenes.scene_blobs(depth=6, sh_degree=2, seed=4, data_seed=5)
    if form == "codebook":
        t0 = po.Tree.from_cells_codebook(s["depth"], 2, s["cells"], s["sigma"], s["sh"], 4096, s["center"],
                                         s["half"])
    else:
        if form == "sg":
            s = dict(s, lobes=scenes.sg_lobes(9, 11))
        t0 = po.Tree.from_scene(s, dtype="f16" if form == "f16" else "f32")
    p = tmp_path / f"{form}.npz"
    t0.save(p, step=3)
    t1, meta = po.Tree.load(p)
    assert int(meta["step"]) == 3 and t1.indexed == t0.indexed
    for a, b in ((t0.child, t1.child), (t0.sigma, t1.sigma), (t0.sh, t1.sh)):
        assert a.dtype == b.dtype and torch.equal(a, b)
    fx, fy, cx, cy = scenes.intrinsics(320, 320, 40.0)
    for W in (96, 320):  # one pass below 65,536 pixels, split above
        cam = po.Camera(scenes.hemisphere_poses(1, 4.0, 9)[0], W, W, fx * W / 320, fy * W / 320, cx * W / 320,
                        cy * W / 320)
        assert torch.equal(po.render_camera(t0, cam), po.render_camera(t1, cam))
    sa, ha = t0.leaf_values()
    sb, hb = t1.leaf_values()
    assert np.array_equal(sa, sb) and np.array_equal(ha, hb)


def test_trainer_resume(po, tmp_path):
    import torch

    _announce("trainer resume")
    gt = scenes.scene_blobs(depth=6, sh_degree=2, seed=4, data_seed=5)
    tgt_tree = po.Tree.from_scene(gt)
    fx, fy, cx, cy = scenes.intrinsics(96, 96, 40.0)
    cams = [po.Camera(p, 96, 96, fx, fy, cx, cy) for p in scenes.hemisphere_poses(12, 4.0, 6)]
    o, d, t = po.optim.training_set(tgt_tree, cams)
    sig, sh = scenes.perturb(gt["sigma"], gt["sh"], 0.3, 8)

    ta = po.Tree.from_cells(gt["depth"], 2, gt["cells"], sig, sh)
    A = po.Trainer(ta, o, d, t, lr_sigma=2e4, lr_sh=1e4, batch=8192, seed=1)
    for _ in range(5):
        A.step()
    p = tmp_path / "fit.npz"
    A.save(p)
    sig5, sh5 = ta.sigma.clone(), ta.sh.clone()
    la = [float(A.step()) for _ in range(5)]

    tb = po.Tree.from_cells(gt["depth"], 2, gt["cells"], sig, sh)
    B = po.Trainer(tb, o, d, t, lr_sigma=2e4, lr_sh=1e4, batch=8192, seed=99)
    B.load(p)
    assert B.steps == 5
    assert torch.equal(tb.sigma, sig5) and torch.equal(tb.sh, sh5)
    lb = [float(B.step()) for _ in range(5)]
    assert B.steps == A.steps == 10
    assert A.seed == B.seed == 1
    # same batches: the gradients differ only by the order of float atomics
    ds = (ta.sigma - tb.sigma).abs().max().item() / ta.sigma.abs().max().item()
    dh = (ta.sh - tb.sh).abs().max().item() / ta.sh.abs().max().item()
    _announce(f"resume: rel diff sigma {ds:.2e} sh {dh:.2e}, losses {la[-1]:.4e} / {lb[-1]:.4e}")
    assert ds < 1e-4 and dh < 1e-4
    assert np.allclose(la, lb, rtol=1e-4)

    # a trainer over another tree refuses the checkpoint
    other = po.Tree.from_scene(scenes.scene_small())
    with pytest.raises(ValueError):
        po.Trainer(other, o, d, t, lr_sigma=1.0, lr_sh=1.0, batch=256).load(p)
