"""Renders through the traversal index (8x8x8 bricks below level D - 3)
against renders through the caller's child array: the same leaves, segments
and arithmetic, so colours, transmittance, sample and cell counts are equal
bit for bit; the index only changes how many child entries a walk reads.
Also the filter weights (atomic max: order independent) and, within float
atomics' reordering, the gradients."""
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


def _say(msg):
    print(f"[gpu] {msg}", file=sys.stderr, flush=True)


def _pair(po, s, dtype="f32"):
    a = po.Tree.from_scene(s, dtype=dtype)
    b = po.Tree.from_scene(s, dtype=dtype, index=False)
    assert a.indexed and not b.indexed
    return a, b


def _scenes():
    mixed = scenes.random_tree_cells(6, 4)
    sig, sh = scenes.leaf_values(len(mixed), 2, 9)
    return {
        "mixed-depth6": dict(depth=6, sh_degree=2, center=(0.0, 0.0, 0.0), half=1.0, cells=mixed, sigma=sig, sh=sh),
        "blobs-depth7": scenes.scene_blobs(depth=7, sh_degree=3, seed=3, data_seed=4),
        "spheres-depth5": scenes.scene_small(),
    }


@pytest.mark.parametrize("name", ["mixed-depth6", "blobs-depth7", "spheres-depth5"])
@pytest.mark.parametrize("dtype", ["f32", "f16"])
def test_index_render_equals_plain_walk(po, name, dtype):
    import torch

    s = _scenes()[name]
    a, b = _pair(po, s, dtype)
    for k, (W, H, one_pass) in enumerate([(96, 80, True), (320, 256, False)]):
        pose = scenes.hemisphere_poses(1, 3.5, 11 + k)[0]
        cam = po.Camera(pose, W, H, *scenes.intrinsics(W, H, 40.0))
        _say(f"{name} {dtype} {W}x{H} one_pass={one_pass}")
        ia, xa = po.render_camera(a, cam, aux=True, one_pass=one_pass)
        ib, xb = po.render_camera(b, cam, aux=True, one_pass=one_pass)
        torch.cuda.synchronize()
        assert torch.equal(ia, ib) and torch.equal(xa, xb)
        sa = po.traversal_stats(a, cam)
        sb = po.traversal_stats(b, cam)
        assert sa["samples"] == sb["samples"] and sa["cells"] == sb["cells"]
        _say(f"  child-entry reads per cell: index {sa['node_loads'] / max(1, sa['cells']):.3f}, "
             f"plain {sb['node_loads'] / max(1, sb['cells']):.3f}")
        if s["depth"] >= 4:
            assert sa["node_loads"] <= sb["node_loads"]
    assert po.device_errors() == 0


def test_index_rays_filter_and_gradients(po):
    import torch

    s = _scenes()["blobs-depth7"]
    a, b = _pair(po, s)
    o, d = scenes.random_rays(70000, 5)
    o = torch.from_numpy(o).cuda()
    d = torch.from_numpy(d).cuda()
    for one_pass in (True, False):
        ra = po.render_rays(a, o, d, one_pass=one_pass)
        rb = po.render_rays(b, o, d, one_pass=one_pass)
        assert torch.equal(ra, rb)
    pose = scenes.hemisphere_poses(1, 3.5, 2)[0]
    cam = po.Camera(pose, 200, 160, *scenes.intrinsics(200, 160, 40.0))
    wa = torch.zeros(a.n_leaves, device="cuda")
    wb = torch.zeros(b.n_leaves, device="cuda")
    po.visibility.leaf_weights(a, [cam], weight=wa)
    po.visibility.leaf_weights(b, [cam], weight=wb)
    assert torch.equal(wa, wb)
    rgb = po.render_rays(a, o, d)
    g = torch.randn_like(rgb)
    ga = po.render_rays_backward(a, o, d, rgb, g)
    gb = po.render_rays_backward(b, o, d, rgb, g)
    torch.cuda.synchronize()
    for x, y in zip(ga, gb):
        scale = float(y.abs().max())
        assert float((x - y).abs().max()) <= 1e-5 * scale
    assert po.device_errors() == 0


def test_index_refuses_a_malformed_tree(po):
    from paper_2103_14024_amd import _lib as L

    s = scenes.scene_small()
    t = po.Tree.from_scene(s, index=False)
    child = t.child.clone()
    child[child > 0] = child.shape[0] + 100
    with pytest.raises(L.PlenOctreeError) as ei:
        po.Tree(s["depth"], s["sh_degree"], child, t.sigma, t.sh)
    assert ei.value.status == L.PO_ERR_TREE
