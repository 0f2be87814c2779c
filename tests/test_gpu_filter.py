"""GPU visibility filter (Sec. 4.2, "Filtering") through the C ABI against
the FP64 oracle: per-leaf maximum ray weight over alpha renders of several
cameras, the alpha maps, the pruning decision and the rebuilt tree.

Tolerance: weights are alphas or contributions of single segments, held to
the render's 1e-4.  With early stopping, a leaf just past a ray's stop point
counts on one side only when the two sides' transmittances straddle the
threshold; the GPU's weights are then checked between the oracle's weights for
thresholds 0.1% above and below (which bracket every ray whose transmittance
error is below 0.1%).
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


def _otree(s, sigma=None, sh=None, cells=None):
    return oracle.OracleTree(s["depth"], s["sh_degree"], s["center"], s["half"],
                             s["cells"] if cells is None else cells,
                             s["sigma"] if sigma is None else sigma, s["sh"] if sh is None else sh)


def _cams(po, n, W, H, radius=3.0, seed=5):
    fx, fy, cx, cy = scenes.intrinsics(W, H, 40.0)
    return [po.Camera(p, W, H, fx, fy, cx, cy) for p in scenes.hemisphere_poses(n, radius, seed)]


def _oracle_rays(cams):
    os_, ds = [], []
    for c in cams:
        f = [float(np.float32(v)) for v in (c.fx, c.fy, c.cx, c.cy)]
        o, d = oracle.camera_rays(np.asarray(c.c2w, np.float32).astype(np.float64), c.width, c.height, *f)
        os_.append(o)
        ds.append(d)
    return np.concatenate(os_), np.concatenate(ds)


def _tree_order(tree, w_caller):
    # oracle weights are in the caller's cell order; the tree's are in leaf order
    return np.asarray(w_caller)[tree.perm]


@pytest.mark.parametrize("dtype", ["f32", "f16"])
@pytest.mark.parametrize("mode", ["alpha", "contrib"])
def test_weights_without_early_stop(po, dtype, mode):
    _announce(f"leaf weights {dtype} {mode}, no early stop")
    s = scenes.scene_small()
    tree = po.Tree.from_scene(s, dtype=dtype)
    sv, hv = tree.leaf_values()
    cams = _cams(po, 6, 48, 40)
    w = po.visibility.leaf_weights(tree, cams, stop_T=0.0, mode=mode).cpu().numpy()
    o, d = _oracle_rays(cams)
    ref = _tree_order(tree, _otree(s, sv, hv).leaf_weights(o, d, gamma=0.0, mode=1 if mode == "contrib" else 0))
    err = np.abs(w - ref)
    _announce(f"max err {err.max():.2e}; leaves met {np.count_nonzero(ref)} of {len(ref)}")
    assert err.max() <= TOL
    assert np.count_nonzero(ref) > 200
    assert po.device_errors() == 0


@pytest.mark.parametrize("mode", ["alpha", "contrib"])
def test_weights_with_early_stop(po, mode):
    _announce(f"leaf weights {mode}, early stop 1e-4")
    s = scenes.scene_small()
    tree = po.Tree.from_scene(s)
    cams = _cams(po, 6, 48, 40)
    H, W = 40, 48
    import torch

    alphas = [torch.empty((H, W), device="cuda") for _ in cams]
    w = po.visibility.leaf_weights(tree, cams, stop_T=1e-4, mode=mode, alpha_out=alphas).cpu().numpy()
    o, d = _oracle_rays(cams)
    ot = _otree(s)
    m = 1 if mode == "contrib" else 0
    hi = _tree_order(tree, ot.leaf_weights(o, d, gamma=1e-4 * 1.001, mode=m))   # stops earlier: fewer segments
    lo = _tree_order(tree, ot.leaf_weights(o, d, gamma=1e-4 * 0.999, mode=m))   # stops later: more segments
    assert np.all(hi <= lo)
    assert np.all(w >= hi - TOL) and np.all(w <= lo + TOL)
    # alpha maps are 1 - T of the camera renders
    _, T, _, _ = ot.render_rays(o, d, gamma=1e-4)
    a = torch.stack(alphas).cpu().numpy().reshape(-1)
    assert np.abs(a - (1.0 - T)).max() <= TOL
    # the maximum does not depend on the order of the cameras
    w2 = po.visibility.leaf_weights(tree, cams[::-1], stop_T=1e-4, mode=mode).cpu().numpy()
    assert np.array_equal(w, w2)


def test_hidden_voxels_and_prune(po):
    import torch

    _announce("opaque wall: hidden layer filtered out, pruned tree renders the same")
    cells, sigma = [], []
    for j in range(8):
        for k in range(8):
            cells += [[3, 2, j, k], [3, 5, j, k]]
            sigma += [1e4, 1.0]
    cells = np.array(cells, np.int32)
    sigma = np.array(sigma, np.float32)
    sig_, sh = scenes.leaf_values(len(cells), 2, 3)
    s = dict(depth=3, sh_degree=2, center=(0.0, 0.0, 0.0), half=1.0, cells=cells, sigma=sigma, sh=sh)
    tree = po.Tree.from_scene(s)
    # cameras on the -x side looking at the wall
    fx, fy, cx, cy = scenes.intrinsics(64, 64, 40.0)
    cams = []
    for y, z in ((0.0, 0.0), (0.4, -0.3), (-0.5, 0.2)):
        pose = scenes.look_at(np.array([-4.0, y, z]), np.array([0.0, 0.0, 0.0]))
        cams.append(po.Camera(pose, 64, 64, fx, fy, cx, cy))
    w = po.visibility.leaf_weights(tree, cams, stop_T=1e-4).cpu().numpy()
    back = np.asarray(sigma)[tree.perm] == 1.0
    assert np.all(w[back] == 0.0)
    assert np.count_nonzero(w[~back] > 0.99) > 20
    pruned, kept = po.visibility.prune(tree, torch.from_numpy(w), 1e-3)
    assert pruned.n_leaves == np.count_nonzero(w >= 1e-3) and not np.any(back[kept])
    for cam in cams:
        a = po.render_camera(tree, cam).cpu().numpy()
        b = po.render_camera(pruned, cam).cpu().numpy()
        assert np.abs(a - b).max() <= TOL


def test_prune_decision_and_rebuilt_tree(po):
    _announce("prune at tau 0.05 against the oracle's weights")
    s = scenes.scene_small()
    tree = po.Tree.from_scene(s)
    cams = _cams(po, 6, 48, 40)
    w = po.visibility.leaf_weights(tree, cams, stop_T=0.0).cpu().numpy()
    o, d = _oracle_rays(cams)
    ref = _tree_order(tree, _otree(s).leaf_weights(o, d, gamma=0.0))
    tau = 0.05
    pruned, kept = po.visibility.prune(tree, w, tau)
    keep = np.zeros(tree.n_leaves, bool)
    keep[kept] = True
    # clear decisions agree with the oracle's; only leaves within the
    # tolerance of the threshold may go either way
    assert np.all(keep[ref >= tau + TOL]) and not np.any(keep[ref < tau - TOL])
    assert 0 < len(kept) < tree.n_leaves
    # the rebuilt tree holds the kept leaves' cells and values and renders as
    # the oracle's tree of those cells
    cells = po.visibility.leaf_cells(tree)
    sig_t = tree.sigma.cpu().numpy()  # tree leaf order
    sh_t = tree.sh[:, :3 * tree.K].cpu().numpy().reshape(-1, 3, tree.K)
    sub = dict(s, cells=cells[kept], sigma=sig_t[kept], sh=sh_t[kept])
    cam = cams[0]
    img = po.render_camera(pruned, cam).cpu().numpy()
    f = [float(np.float32(v)) for v in (cam.fx, cam.fy, cam.cx, cam.cy)]
    ref_img, _, _ = _otree(sub).render_camera(np.asarray(cam.c2w, np.float32), cam.width, cam.height, *f,
                                              gamma=1e-4)
    assert np.abs(img - ref_img).max() <= TOL
