"""Direct octree optimisation (Sec. 4.3) through the library kernels: loss
gradient and SGD kernels against their definitions, and a short run whose
loss falls.  The trajectory itself is not pinned (atomic summation order)."""
import sys

import numpy as np
import pytest

from paper_2103_14024_amd import scenes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def po():
    import torch

    assert torch.cuda.is_available()
    import paper_2103_14024_amd as po

    return po


def test_camera_rays_match_definition(po):
    import torch

    W, H = 37, 21
    pose = scenes.small_pose()
    fx, fy, cx, cy = scenes.intrinsics(W, H, 40.0)
    o, d = po.camera_rays(po.Camera(pose, W, H, fx, fy, cx, cy))
    v, u = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    cam = np.stack([(u + 0.5 - cx) / fx, -(v + 0.5 - cy) / fy, -np.ones_like(u, dtype=np.float64)], -1)
    ref = cam.reshape(-1, 3) @ np.asarray(pose, np.float64)[:, :3].T
    ref /= np.linalg.norm(ref, axis=1, keepdims=True)
    assert np.abs(d.cpu().numpy() - ref).max() < 1e-6
    assert np.all(o.cpu().numpy() == np.asarray(pose, np.float32)[:, 3])


def test_loss_grad_and_sgd_kernels(po):
    import ctypes

    import torch

    from paper_2103_14024_amd import _lib as L

    n = 10007
    g = torch.Generator(device="cuda").manual_seed(0)
    rgb = torch.rand((n, 3), device="cuda", generator=g)
    tgt = torch.rand((n, 3), device="cuda", generator=g)
    grad = torch.empty_like(rgb)
    sq = torch.zeros(1, device="cuda")
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    L.call("po_mse_grad", n, rgb.data_ptr(), tgt.data_ptr(), ctypes.c_float(1.0 / (3 * n)), grad.data_ptr(),
           sq.data_ptr(), s)
    e = (rgb - tgt).double()
    assert torch.allclose(grad.double(), 2 * e / (3 * n), rtol=1e-6, atol=1e-12)
    assert abs(sq.item() - float((e ** 2).sum())) < 1e-4 * float((e ** 2).sum())
    p = torch.rand(5003, device="cuda", generator=g)
    gp = torch.rand(5003, device="cuda", generator=g)
    want = p - 0.25 * gp
    L.call("po_sgd_step", 5003, p.data_ptr(), gp.data_ptr(), ctypes.c_float(0.25), 1, s)
    assert torch.allclose(p, want, rtol=1e-6, atol=1e-7) and gp.abs().max().item() == 0.0
    # zero gradients and signed zeros: p - lr g bit for bit (lr a power of
    # two, so the product is exact and the float32 subtraction rounds once,
    # as the fused multiply-add does)
    m = 4099
    p = torch.rand(m, device="cuda", generator=g) - 0.5
    gp = torch.rand(m, device="cuda", generator=g) - 0.5
    p[::3] = 0.0
    p[1::3] = -0.0
    gp[::2] = 0.0
    gp[1::4] = -0.0
    want = (p.cpu() - 0.25 * gp.cpu()).view(torch.int32)
    L.call("po_sgd_step", m, p.data_ptr(), gp.data_ptr(), ctypes.c_float(0.25), 1, s)
    torch.cuda.synchronize()
    assert torch.equal(p.cpu().view(torch.int32), want)
    assert int((gp.view(torch.int32) != 0).sum()) == 0  # every gradient cleared to +0


def test_draw_batch(po):
    # the device draw against the SplitMix64 reference: the same rows, and
    # the loss accumulator cleared
    import ctypes

    import torch

    from paper_2103_14024_amd import _lib as L
    from splitmix import draw_rows

    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    g = torch.Generator(device="cuda").manual_seed(5)
    n_src, n = 123_457, 10_007
    o, d, t = (torch.rand((n_src, 3), device="cuda", generator=g) for _ in range(3))
    bo, bd, bt = (torch.empty((n, 3), device="cuda") for _ in range(3))
    sq = torch.full((1,), 5.0, device="cuda")
    seed, first = 0xDEADBEEF12345678, 3 * n
    L.call("po_draw_batch", n, ctypes.c_uint64(seed), ctypes.c_uint64(first), n_src, o.data_ptr(), d.data_ptr(),
           t.data_ptr(), bo.data_ptr(), bd.data_ptr(), bt.data_ptr(), sq.data_ptr(), s)
    torch.cuda.synchronize()
    idx = torch.tensor(draw_rows(seed, first, n, n_src), device="cuda")
    assert torch.equal(bo, o[idx]) and torch.equal(bd, d[idx]) and torch.equal(bt, t[idx])
    assert sq.item() == 0.0
    # no accumulator: nothing else written; n = 0 does nothing
    L.call("po_draw_batch", 5, ctypes.c_uint64(1), ctypes.c_uint64(0), n_src, o.data_ptr(), d.data_ptr(),
           t.data_ptr(), bo.data_ptr(), bd.data_ptr(), bt.data_ptr(), None, s)
    L.call("po_draw_batch", 0, ctypes.c_uint64(1), ctypes.c_uint64(0), n_src, None, None, None, None, None, None,
           None, s)
    torch.cuda.synchronize()
    assert torch.equal(bo[:5], o[torch.tensor(draw_rows(1, 0, 5, n_src), device="cuda")])
    with pytest.raises(L.PlenOctreeError):
        L.call("po_draw_batch", 5, ctypes.c_uint64(1), ctypes.c_uint64(0), 0, o.data_ptr(), d.data_ptr(),
               t.data_ptr(), bo.data_ptr(), bd.data_ptr(), bt.data_ptr(), None, s)


def test_loss_grad_large_and_gather(po):
    # the loss gradient over more rays than one grid pass covers (grid-stride
    # loop, one atomic per workgroup) and the batch gather against its
    # definition, including an out-of-range index (zeros, counted)
    import ctypes

    import torch

    from paper_2103_14024_amd import _lib as L

    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    g = torch.Generator(device="cuda").manual_seed(3)
    n = 400_003
    rgb = torch.rand((n, 3), device="cuda", generator=g)
    tgt = torch.rand((n, 3), device="cuda", generator=g)
    grad = torch.empty_like(rgb)
    sq = torch.zeros(1, device="cuda")
    L.call("po_mse_grad", n, rgb.data_ptr(), tgt.data_ptr(), ctypes.c_float(1.0 / (3 * n)), grad.data_ptr(),
           sq.data_ptr(), s)
    e = (rgb - tgt).double()
    assert torch.allclose(grad.double(), 2 * e / (3 * n), rtol=1e-6, atol=1e-14)
    assert abs(sq.item() - float((e ** 2).sum())) < 1e-5 * float((e ** 2).sum())
    m, k = 50_000, 7001
    o, d, t = (torch.rand((m, 3), device="cuda", generator=g) for _ in range(3))
    idx = torch.randint(0, m, (k,), device="cuda", generator=g)
    idx[5] = m  # out of range
    bo, bd, bt = (torch.full((k, 3), 7.0, device="cuda") for _ in range(3))
    po.reset_device_errors()
    L.call("po_gather_rays", k, idx.data_ptr(), m, o.data_ptr(), d.data_ptr(), t.data_ptr(), bo.data_ptr(),
           bd.data_ptr(), bt.data_ptr(), s)
    ok = torch.ones(k, dtype=torch.bool, device="cuda")
    ok[5] = False
    for src, dst in ((o, bo), (d, bd), (t, bt)):
        assert torch.equal(dst[ok], src[idx[ok]])
        assert torch.equal(dst[5], torch.zeros(3, device="cuda"))
    assert po.device_errors() == 1
    po.reset_device_errors()
    with pytest.raises(L.PlenOctreeError):
        L.call("po_gather_rays", k, idx.data_ptr(), 0, o.data_ptr(), d.data_ptr(), t.data_ptr(), bo.data_ptr(),
               bd.data_ptr(), bt.data_ptr(), s)


def test_training_reduces_loss(po):
    gt = scenes.scene_blobs(depth=6, sh_degree=2, seed=4, data_seed=5)
    tgt_tree = po.Tree.from_scene(gt)
    fx, fy, cx, cy = scenes.intrinsics(96, 96, 40.0)
    cams = [po.Camera(p, 96, 96, fx, fy, cx, cy) for p in scenes.hemisphere_poses(12, 4.0, 6)]
    o, d, t = po.optim.training_set(tgt_tree, cams)
    sig, sh = scenes.perturb(gt["sigma"], gt["sh"], 0.3, 8)
    tree = po.Tree.from_cells(gt["depth"], 2, gt["cells"], sig, sh)
    m0 = po.optim.dataset_mse(tree, o, d, t)
    tr = po.Trainer(tree, o, d, t, lr_sigma=2e4, lr_sh=2e4, batch=8192, seed=1)
    losses = [float(tr.step()) for _ in range(150)]
    m1 = po.optim.dataset_mse(tree, o, d, t)
    print(f"[gpu] train: dataset mse {m0:.3e} -> {m1:.3e}, batch loss {np.mean(losses[:10]):.3e} -> "
          f"{np.mean(losses[-10:]):.3e}", file=sys.stderr, flush=True)
    assert m1 < 0.5 * m0
    assert np.mean(losses[-10:]) < np.mean(losses[:10])


def test_trainer_step_matches_oracle_update(po):
    # one Trainer step (65536-ray batch: the split backward) with distinct
    # learning rates for densities and coefficients, on its own stream: the
    # parameter change divided by each learning rate must be the FP64 oracle
    # gradient of the mean squared error over the batch (threshold-straddle
    # rule at stop_T), and the gradient buffers are cleared by the step
    import torch

    import gradcheck
    import oracle

    gt = scenes.scene_blobs(depth=6, sh_degree=2, seed=4, data_seed=5)
    tgt_tree = po.Tree.from_scene(gt)
    fx, fy, cx, cy = scenes.intrinsics(96, 96, 40.0)
    cams = [po.Camera(p, 96, 96, fx, fy, cx, cy) for p in scenes.hemisphere_poses(12, 4.0, 6)]
    o, d, t = po.optim.training_set(tgt_tree, cams)
    sig, sh = scenes.perturb(gt["sigma"], gt["sh"], 0.3, 8)
    tree = po.Tree.from_cells(gt["depth"], 2, gt["cells"], sig, sh)
    sig0 = tree.sigma.detach().clone()
    sh0 = tree.sh.detach().clone()
    lr_s, lr_h = 1.0e7, 2.5e6
    tr = po.Trainer(tree, o, d, t, lr_sigma=lr_s, lr_sh=lr_h, batch=65536, seed=3)
    stream = torch.cuda.Stream()
    loss = tr.step(stream=stream)
    stream.synchronize()
    # the batch the step drew, its forward colours and upstream gradient
    bo, bd = tr.bo.cpu().numpy(), tr.bd.cpu().numpy()
    rgb, bt = tr.rgb.cpu().numpy().astype(np.float64), tr.bt.cpu().numpy().astype(np.float64)
    g = tr.grad_rgb.cpu().numpy().astype(np.float64)
    n = tr.batch
    assert np.allclose(g, 2.0 * (rgb - bt) / (3 * n), rtol=1e-6, atol=1e-15)
    assert abs(float(loss) - float(((rgb - bt) ** 2).mean())) <= 1e-5 * float(((rgb - bt) ** 2).mean())
    assert float(tr.g_sigma.abs().max()) == 0.0 and float(tr.g_sh.abs().max()) == 0.0
    ot = oracle.OracleTree(gt["depth"], 2, gt["center"], gt["half"], gt["cells"], sig, sh)
    (ls, hs), (lh, hh), n_str = gradcheck.grad_envelope(ot, bo, bd, g, (1.0, 1.0, 1.0), 1e-4)
    print(f"[gpu] trainer step: {n_str} straddling rays", file=sys.stderr, flush=True)
    # p' = fl(p - lr g): the change over lr carries half an ulp of p' over lr
    s1, h1 = tree.sigma.detach().double().cpu().numpy(), tree.sh.detach().double().cpu().numpy()
    s0, h0 = sig0.double().cpu().numpy(), sh0.double().cpu().numpy()
    est_s, est_h = gradcheck.to_cells(tree, (s0 - s1) / lr_s, (h0 - h1) / lr_h)
    ulp_s, ulp_h = gradcheck.to_cells(tree, np.spacing(np.abs(s1).astype(np.float32)) / lr_s,
                                      np.spacing(np.abs(h1).astype(np.float32)) / lr_h)
    K = tree.K
    # padding columns of the records are not touched
    assert np.array_equal(h1[:, 3 * K:], h0[:, 3 * K:])
    gradcheck.check(est_s, ls, hs, "trainer step dsigma", slack=0.5 * ulp_s)
    gradcheck.check(est_h, lh, hh, "trainer step dsh", slack=0.5 * ulp_h)
