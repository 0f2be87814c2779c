"""GPU viewer outputs (Sec. 5.5, "Interactive demos") through the C ABI
against the FP64 oracle: depth map, alpha map (1 - T), SH-component subsets
and slicing planes, on the ray and camera paths and in batched launches.

Tolerances: colour and transmittance 1e-4 absolute, the bar of every render.
The depth is a sum of weights times distances; its error is at most the
weights' error (the colour bar) times the largest distance to the box, so it
is compared within 1e-4 * (|o| + box diagonal) per ray.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2103_14024_amd import scenes

pytestmark = pytest.mark.gpu
TOL = 1e-4
DIAG = 2.0 * np.sqrt(3.0)


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


def _otree(s, sigma=None, sh=None):
    return oracle.OracleTree(s["depth"], s["sh_degree"], s["center"], s["half"], s["cells"],
                             s["sigma"] if sigma is None else sigma, s["sh"] if sh is None else sh)


def _rays():
    o1, d1 = scenes.random_rays(4096 + 37, 21)
    o2, d2 = scenes.inside_rays(300, 22)
    o3 = np.array([[-3.0, 0.0, 0.25], [0.5, -3.0, -0.5], [0.0, 0.0, 3.0], [-3.0, -0.125, 0.0625]], np.float32)
    d3 = np.array([[1, 0, 0], [0, 1, 0], [0, 0, -1], [1, 0.0, 0.0]], np.float32)
    return np.concatenate([o1, o2, o3]), np.concatenate([d1, d2, d3])


def _depth_tol(o):
    return TOL * (np.linalg.norm(np.asarray(o, np.float64), axis=1) + DIAG)


def _check(tag, rgb, aux, ref, o):
    rr, T, ns, dep = ref
    e_rgb = np.abs(rgb - rr).max()
    e_T = np.abs(aux[:, 0] - T).max()
    e_d = np.abs(aux[:, 3] - dep)
    _announce(f"{tag}: rgb {e_rgb:.2e} T {e_T:.2e} depth {e_d.max():.2e} (rel {np.max(e_d / _depth_tol(o)):.2f} of tol)")
    assert e_rgb <= TOL, tag
    assert e_T <= TOL, tag
    assert np.all(e_d <= _depth_tol(o)), tag
    # sample counts agree except where a corner-clipped segment rounds to zero length
    assert np.mean(aux[:, 1] == ns) > 0.99 and np.abs(aux[:, 1] - ns).max() <= 2, tag


def test_aux_does_not_change_colour(po):
    # the viewer kernels composite exactly as the plain ones
    _announce("viewer kernel colours equal plain kernel colours")
    s = scenes.scene_small()
    tree = po.Tree.from_scene(s)
    o, d = _rays()
    c0 = po.render_rays(tree, _dev(o), _dev(d)).cpu().numpy()
    c1, aux = po.render_rays(tree, _dev(o), _dev(d), aux=True)
    assert np.array_equal(c0, c1.cpu().numpy())
    cam = po.Camera(scenes.small_pose(), 72, 40, *scenes.intrinsics(72, 40, 40.0))
    i0 = po.render_camera(tree, cam).cpu().numpy()
    i1, _ = po.render_camera(tree, cam, aux=True)
    assert np.array_equal(i0, i1.cpu().numpy())


@pytest.mark.parametrize("dtype", ["f32", "f16"])
@pytest.mark.parametrize("stop_T", [0.0, 1e-4])
def test_depth_and_alpha(po, dtype, stop_T):
    _announce(f"depth and alpha, {dtype}, stop_T {stop_T}")
    s = scenes.scene_small()
    tree = po.Tree.from_scene(s, dtype=dtype)
    sv, hv = tree.leaf_values()
    o, d = _rays()
    rgb, aux = po.render_rays(tree, _dev(o), _dev(d), stop_T=stop_T, aux=True)
    ref = _otree(s, sv, hv).render_view(o, d, gamma=stop_T)
    _check(f"depth {dtype} {stop_T}", rgb.cpu().numpy(), aux.cpu().numpy(), ref, o)
    assert ref[3].max() > 1.0  # rays do terminate inside the scene


def test_sh_subsets(po):
    s = scenes.scene_small()
    tree = po.Tree.from_scene(s)
    ot = _otree(s)
    o, d = _rays()
    for off in (0b1, 0b110, 0b111111110, 0b111110000, (1 << 9) - 1, 1 << 20):
        _announce(f"sh_off {off:#x}")
        rgb, aux = po.render_rays(tree, _dev(o), _dev(d), aux=True, sh_off=off)
        _check(f"sh_off {off:#x}", rgb.cpu().numpy(), aux.cpu().numpy(),
               ot.render_view(o, d, gamma=1e-4, sh_off=off), o)


PLANES = [
    (1.0, 0.0, 0.0, 0.0),         # grid plane through the centre, keep x >= 0
    (0.0, -1.0, 0.0, 0.25),       # keep y <= 0.25 (off the grid planes of coarse levels)
    (0.3, -0.5, 0.8, -0.1),       # oblique
    (0.0, 0.0, 0.0, 1.0),         # keeps everything
    (0.0, 0.0, 0.0, -1.0),        # keeps nothing
    (0.0, 0.0, 2.0, 5.0),         # the whole box is inside: no cut
]


@pytest.mark.parametrize("plane", PLANES)
def test_slicing_plane(po, plane):
    _announce(f"slicing plane {plane}")
    s = scenes.scene_small()
    tree = po.Tree.from_scene(s)
    o, d = _rays()
    rgb, aux = po.render_rays(tree, _dev(o), _dev(d), aux=True, clip=plane)
    ref = _otree(s).render_view(o, d, gamma=1e-4, clip=np.asarray(plane, np.float32))
    _check(f"clip {plane}", rgb.cpu().numpy(), aux.cpu().numpy(), ref, o)
    if plane == (0.0, 0.0, 0.0, -1.0):
        assert np.all(rgb.cpu().numpy() == 1.0)


def test_camera_and_batch(po):
    import torch

    s = scenes.scene_small()
    tree = po.Tree.from_scene(s)
    pose = scenes.small_pose()
    W, H = 72, 40
    fx, fy, cx, cy = scenes.intrinsics(W, H, 40.0)
    cam = po.Camera(pose, W, H, fx, fy, cx, cy)
    plane = (0.2, 0.9, -0.3, 0.05)
    off = 0b000001110
    _announce("camera with depth, SH subset and slicing plane")
    img, aux = po.render_camera(tree, cam, aux=True, sh_off=off, clip=plane)
    f32 = [float(np.float32(v)) for v in (fx, fy, cx, cy)]  # the camera carries float32 intrinsics
    o, d = oracle.camera_rays(np.asarray(pose, np.float32).astype(np.float64), W, H, *f32)
    ref = _otree(s).render_view(o, d, gamma=1e-4, sh_off=off, clip=np.asarray(plane, np.float32))
    _check("camera view", img.cpu().numpy().reshape(-1, 3), aux.cpu().numpy().reshape(-1, 4), ref, o)
    # a batch mixing viewer and plain jobs renders each as alone
    _announce("batch mixing viewer and plain jobs")
    outs = [torch.empty((H, W, 3), device="cuda") for _ in range(3)]
    a0 = torch.empty((H, W, 4), device="cuda")
    jobs = [po.Job(tree, cam, outs[0], aux_out=a0, sh_off=off, clip=plane),
            po.Job(tree, cam, outs[1]),
            po.Job(tree, cam, outs[2], clip=plane)]
    po.render_batch(jobs)
    torch.cuda.synchronize()
    assert torch.equal(outs[0], img) and torch.equal(a0, aux)
    assert torch.equal(outs[1], po.render_camera(tree, cam))
    assert torch.equal(outs[2], po.render_camera(tree, cam, clip=plane))
    assert po.device_errors() == 0
