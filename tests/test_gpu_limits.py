"""GPU renders at the limits the ABI accepts, against the FP64 oracle: the
maximum tree depth (15) and the maximum image size (16384 x 16384), checked
on pixel windows at the image's corners and centre (the oracle traces the
same pixels through a shifted principal point, which is exact in FP64)."""
import sys

import numpy as np
import pytest

import oracle
from paper_2103_14024_amd import scenes

pytestmark = pytest.mark.gpu
TOL = 1e-4


@pytest.fixture(scope="module")
def po():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2103_14024_amd as po

    po.reset_device_errors()
    return po


def _announce(msg):
    print(f"[gpu] {msg}", file=sys.stderr, flush=True)


def _dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, np.float32))).cuda()


def test_max_depth(po):
    from paper_2103_14024_amd import _lib as L

    depth = L.PO_MAX_DEPTH
    _announce(f"depth {depth} tree")
    rng = np.random.default_rng(15)
    # a dense 12^3 cluster of finest leaves near the box centre, plus coarse leaves elsewhere
    base = (1 << depth) // 2 - 6
    g = np.stack(np.meshgrid(*[np.arange(12)] * 3, indexing="ij"), -1).reshape(-1, 3) + base
    fine = np.column_stack([np.full(len(g), depth), g])
    coarse = np.array([[3, 0, 0, 0], [3, 7, 7, 7], [2, 0, 3, 1], [4, 15, 2, 9]])
    cells = np.concatenate([fine, coarse]).astype(np.int32)
    sigma, sh = scenes.leaf_values(len(cells), 2, 16, mu=8.0, s=0.5)  # thin cells need high density
    s = dict(depth=depth, sh_degree=2, center=(0.25, -0.5, 0.125), half=1.5, cells=cells, sigma=sigma, sh=sh)
    tree = po.Tree.from_scene(s)
    ot = oracle.OracleTree(depth, 2, s["center"], s["half"], cells, sigma, sh)
    # rays aimed at the cluster from random directions, and free rays
    c = np.array(s["center"]) + (base + 6 - (1 << depth) / 2) * (2 * s["half"] / (1 << depth))
    v = rng.standard_normal((3000, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    tgt = c + rng.uniform(-1, 1, (3000, 3)) * 10 * (2 * s["half"] / (1 << depth))
    o1 = (tgt + 3.0 * v).astype(np.float32)
    d1 = (tgt - o1).astype(np.float32)
    o2, d2 = scenes.random_rays(1000, 17, radius=4.0, spread=1.6)
    o = np.concatenate([o1, o2])
    d = np.concatenate([d1, d2])
    rgb, aux = po.render_rays(tree, _dev(o), _dev(d), bg=(0.2, 0.5, 0.9), aux=True)
    ref, T, ns, _ = ot.render_rays(o, d, bg=(0.2, 0.5, 0.9), gamma=1e-4)
    err = np.abs(rgb.cpu().numpy() - ref)
    _announce(f"depth {depth}: max err {err.max():.2e}; rays with samples {np.count_nonzero(ns)}; max samples {ns.max()}")
    assert err.max() <= TOL
    assert np.count_nonzero(ns > 5) > 500
    assert po.device_errors() == 0


def test_max_image_size(po):
    import torch

    from paper_2103_14024_amd import _lib as L

    W = H = 16384
    _announce(f"{W}x{H} image")
    s = scenes.scene_small()
    tree = po.Tree.from_scene(s)
    pose = scenes.small_pose()
    fx, fy, cx, cy = scenes.intrinsics(W, H, 40.0)
    cam = po.Camera(pose, W, H, fx, fy, cx, cy)
    img = po.render_camera(tree, cam)
    torch.cuda.synchronize()
    ot = oracle.OracleTree(s["depth"], s["sh_degree"], s["center"], s["half"], s["cells"], s["sigma"], s["sh"])
    f32 = [float(np.float32(v)) for v in (fx, fy, cx, cy)]
    for x0, y0 in ((0, 0), (W - 8, 0), (0, H - 8), (W - 8, H - 8), (W // 2 - 4, H // 2 - 4), (5000, 11000)):
        o, d = oracle.camera_rays(np.asarray(pose, np.float32).astype(np.float64), 8, 8, f32[0], f32[1],
                                  f32[2] - x0, f32[3] - y0)
        ref, _, _, _ = ot.render_rays(o, d, gamma=1e-4)
        got = img[y0:y0 + 8, x0:x0 + 8].cpu().numpy().reshape(-1, 3)
        assert np.abs(got - ref).max() <= TOL, (x0, y0)
    # the scene is visible in the middle of the image
    assert float((img[H // 2 - 64:H // 2 + 64, W // 2 - 64:W // 2 + 64] - 1.0).abs().max()) > 0.05
    del img
    torch.cuda.empty_cache()
    # one pixel more is refused
    big = po.Camera(pose, W + 1, 8, fx, fy, cx, cy)
    with pytest.raises(po.PlenOctreeError):
        po.render_camera(tree, big)
    assert L.PO_TILE == 16
    assert po.device_errors() == 0
