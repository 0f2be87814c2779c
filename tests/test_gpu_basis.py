"""GPU colour-basis variants (App. A basis ablation, App. B.1) through the C
ABI against the FP64 oracle: SH degree 4 (SH-25) and spherical Gaussians with
per-tree lobes (SG-9/16/25), for renders, the viewer's basis subsets,
gradients and batches that mix SH and SG trees.

Bars as for the other renders and gradients: colour 1e-4 absolute; gradients
max error <= 1e-4 of the largest reference value and cosine >= 0.99999.
"""
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


def _scene(deg, sg, seed=1):
    s = scenes.scene_small(data_seed=seed, sh_degree=deg)
    if sg:
        s["lobes"] = scenes.sg_lobes((deg + 1) ** 2, seed + 7)
    return s


def _otree(s, sigma=None, sh=None):
    return oracle.OracleTree(s["depth"], s["sh_degree"], s["center"], s["half"], s["cells"],
                             s["sigma"] if sigma is None else sigma, s["sh"] if sh is None else sh,
                             lobes=s.get("lobes"))


def _rays():
    o1, d1 = scenes.random_rays(4096 + 37, 41)
    o2, d2 = scenes.inside_rays(300, 42)
    return np.concatenate([o1, o2]), np.concatenate([d1, d2])


CASES = [(4, False), (2, True), (3, True), (4, True)]


@pytest.mark.parametrize("dtype", ["f32", "f16"])
@pytest.mark.parametrize("deg,sg", CASES)
def test_render_parity(po, deg, sg, dtype):
    tag = f"{'SG' if sg else 'SH'}-{(deg + 1) ** 2} {dtype}"
    _announce(f"render {tag}")
    s = _scene(deg, sg)
    tree = po.Tree.from_scene(s, dtype=dtype)
    sv, hv = tree.leaf_values()
    ot = _otree(s, sv, hv)
    o, d = _rays()
    rgb = po.render_rays(tree, _dev(o), _dev(d)).cpu().numpy()
    ref, _, ns, _ = ot.render_rays(o, d, gamma=1e-4)
    err = np.abs(rgb - ref).max()
    _announce(f"{tag}: rays max err {err:.2e}")
    assert err <= TOL and ns.max() > 0
    # camera path and a basis subset through the viewer kernels
    pose = scenes.small_pose()
    W, H = 40, 24
    fx, fy, cx, cy = scenes.intrinsics(W, H, 40.0)
    cam = po.Camera(pose, W, H, fx, fy, cx, cy)
    img = po.render_camera(tree, cam).cpu().numpy()
    f32 = [float(np.float32(v)) for v in (fx, fy, cx, cy)]
    ref_img, _, _ = ot.render_camera(np.asarray(pose, np.float32), W, H, *f32, gamma=1e-4)
    assert np.abs(img - ref_img).max() <= TOL
    off = 0b1011000110
    rgb, aux = po.render_rays(tree, _dev(o), _dev(d), aux=True, sh_off=off)
    ref, T, _, dep = ot.render_view(o, d, gamma=1e-4, sh_off=off)
    assert np.abs(rgb.cpu().numpy() - ref).max() <= TOL
    assert po.device_errors() == 0


def _compare(got, ref, what):
    scale = np.abs(ref).max()
    err = np.abs(got - ref).max()
    cos = float((got * ref).sum() / (np.linalg.norm(got) * np.linalg.norm(ref) + 1e-300))
    _announce(f"{what}: max|ref| {scale:.3e} rel err {err / scale:.2e} cos {cos:.8f}")
    assert err <= 1e-4 * scale, what
    assert cos >= 0.99999, what


@pytest.mark.parametrize("deg,sg", [(4, False), (2, True), (4, True)])
def test_backward_parity(po, deg, sg):
    s = _scene(deg, sg, seed=3)
    s["sigma"] = s["sigma"].copy()
    s["sigma"][::7] *= -1.0
    tree = po.Tree.from_scene(s)
    o, d = scenes.random_rays(4000, 9, spread=1.0)
    g = np.random.default_rng(4).standard_normal((len(o), 3)).astype(np.float32)
    bg = (0.9, 0.4, 0.1)
    rgb = po.render_rays(tree, _dev(o), _dev(d), bg=bg)
    gs, gsh = po.render_rays_backward(tree, _dev(o), _dev(d), rgb, _dev(g), bg=bg)
    K = tree.K
    a = np.zeros(tree.n_leaves)
    b = np.zeros((tree.n_leaves, 3 * K))
    a[tree.perm] = gs.cpu().numpy()
    b[tree.perm] = gsh.cpu().numpy()[:, :3 * K]
    rs, rsh = _otree(s).grad(o, d, g, bg=bg, gamma=1e-4)
    tag = f"{'SG' if sg else 'SH'}-{K}"
    _compare(a, rs, f"dsigma {tag}")
    _compare(b.reshape(-1, 3, K), rsh, f"dsh {tag}")


def test_batch_mixes_sh_and_sg(po):
    import torch

    _announce("batch with SH and SG trees of the same K")
    t_sh = po.Tree.from_scene(_scene(3, False))
    t_sg = po.Tree.from_scene(_scene(3, True))
    pose = scenes.small_pose()
    W, H = 48, 32
    cam = po.Camera(pose, W, H, *scenes.intrinsics(W, H, 40.0))
    outs = [torch.empty((H, W, 3), device="cuda") for _ in range(2)]
    po.render_batch([po.Job(t_sg, cam, outs[0]), po.Job(t_sh, cam, outs[1])])
    torch.cuda.synchronize()
    assert torch.equal(outs[0], po.render_camera(t_sg, cam))
    assert torch.equal(outs[1], po.render_camera(t_sh, cam))
    assert not torch.equal(outs[0], outs[1])
