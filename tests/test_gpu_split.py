"""The split render and the split backward against the one-pass kernels and
the FP64 oracle.

Camera renders of 2^16 pixels or more (and ray lists and backward passes of
2^16 rays or more) walk every ray for a bounded number of cells, hand the
rays with cells left on as pieces walked in parallel, and join the piece
results front to back (Sec. 3, eqn:quad: the composite of a range of segments
acts on what lies behind it through its colour and transmittance).  Where
early stopping ends a ray inside a piece, the join walks that piece again
from the known transmittance.  Covered: every compiled K, SG, float16 and
codebook leaves, the viewer outputs, ray lists, the depth-15 tree, queue
overflow, queue release and a second stream, and the gradients (App. B.3).

The scene is a ball of fog: finest cells of moderate density, so that rays
through its middle walk a hundred cells or more and reach T < 1e-4 deep inside
(the chunk walked again), while rays near its rim leave it first.  The
one-pass render of the same pixels comes from render_batch with one_pass
set.  The two differ by float rounding only; where T lands within rounding
of stop_T the two may stop one cell apart, which moves at most T = stop_T of
weight.
"""
import sys

import numpy as np
import pytest

import gradcheck
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


def _say(msg):
    print(f"[gpu] {msg}", file=sys.stderr, flush=True)


def fog_scene(depth=7, radius=0.8, sh_degree=1, seed=31):
    """Every finest cell whose centre lies in a ball, sigma ~ U(4, 10)."""
    n = 1 << depth
    c = (np.arange(n) + 0.5) * (2.0 / n) - 1.0
    x, y, z = np.meshgrid(c, c, c, indexing="ij")
    ijk = np.argwhere(x * x + y * y + z * z <= radius * radius).astype(np.int32)
    cells = np.column_stack([np.full(len(ijk), depth, np.int32), ijk])
    rng = np.random.default_rng(seed)
    K = (sh_degree + 1) ** 2
    sigma = rng.uniform(4.0, 10.0, len(cells)).astype(np.float32)
    sh = rng.normal(0.0, 0.5, (len(cells), 3, K)).astype(np.float32)
    return dict(depth=depth, sh_degree=sh_degree, center=(0.0, 0.0, 0.0), half=1.0, cells=cells, sigma=sigma, sh=sh)


@pytest.fixture(scope="module")
def fog(po):
    s = fog_scene()
    _say(f"fog ball: {len(s['cells'])} leaves")
    tree = po.Tree.from_scene(s)
    ot = oracle.OracleTree(s["depth"], s["sh_degree"], s["center"], s["half"], s["cells"], s["sigma"], s["sh"])
    return s, tree, ot


def _cam(po, W, H, seed=3, radius=2.6, fov=40.0):
    pose = scenes.hemisphere_poses(1, radius, seed)[0]
    return po.Camera(pose, W, H, *scenes.intrinsics(W, H, fov)), pose


def _one_pass(po, tree, cam, stop_T, aux=False):
    import torch

    out = torch.empty((cam.height, cam.width, 3), device="cuda")
    a = torch.empty((cam.height, cam.width, 4), device="cuda") if aux else None
    po.render_batch([po.Job(tree, cam, out, stop_T=stop_T, aux_out=a, one_pass=True)])
    torch.cuda.synchronize()
    return out.cpu().numpy(), (a.cpu().numpy() if aux else None)


def _oracle_pixels(ot, cam, pose, idx, stop_T):
    f32 = [float(np.float32(v)) for v in (cam.fx, cam.fy, cam.cx, cam.cy)]
    o, d = oracle.camera_rays(np.asarray(pose, np.float32).astype(np.float64), cam.width, cam.height, *f32)
    ref, T, ns, _ = ot.render_rays(o[idx], d[idx], gamma=stop_T)
    return ref, T


@pytest.mark.parametrize("stop_T", [0.0, 1e-4])
def test_split_matches_oracle_and_one_pass(po, fog, stop_T):
    s, tree, ot = fog
    W = H = 256
    cam, pose = _cam(po, W, H)
    _say(f"split render {W}x{H}, stop_T {stop_T}")
    img = po.render_camera(tree, cam, stop_T=stop_T).cpu().numpy()
    one, aux = _one_pass(po, tree, cam, stop_T, aux=True)
    steps, T = aux[..., 2].reshape(-1), aux[..., 0].reshape(-1)
    long_rays = steps > 32
    stopped_late = long_rays & (T < stop_T)
    _say(f"rays past 32 cells: {long_rays.sum()}, of which stopped: {stopped_late.sum()}; max steps {steps.max():.0f}")
    assert long_rays.sum() > 15000
    if stop_T > 0:
        # early stopping inside the handed-on part of many rays
        assert stopped_late.sum() > 5000
    d = np.abs(img - one).max(-1).reshape(-1)
    _say(f"split vs one pass: max {d.max():.2e}, pixels above 1e-5: {(d > 1e-5).sum()}")
    assert np.mean(d > 1e-5) <= 1e-4 and d.max() <= stop_T + 1e-5
    # oracle: random pixels and the longest walks
    rng = np.random.default_rng(7)
    idx = np.unique(np.concatenate([rng.choice(W * H, 2000, replace=False), np.argsort(-steps)[:300]]))
    ref, Tref = _oracle_pixels(ot, cam, pose, idx, stop_T)
    err = np.abs(img.reshape(-1, 3)[idx] - ref).max(1)
    _say(f"split vs oracle on {len(idx)} pixels: max {err.max():.2e} mean {err.mean():.2e}")
    assert err.max() <= TOL
    if stop_T > 0:
        assert np.sum(Tref < stop_T) > 300
    assert po.device_errors() == 0


def test_split_early_stop_near_one_percent(po, fog):
    # stop_T = 1e-2 (the paper's threshold): stops come early in most walks
    s, tree, ot = fog
    cam, pose = _cam(po, 320, 240, seed=5)
    img = po.render_camera(tree, cam, stop_T=1e-2).cpu().numpy()
    one, _ = _one_pass(po, tree, cam, 1e-2)
    d = np.abs(img - one).max(-1)
    _say(f"stop_T 1e-2: split vs one pass max {d.max():.2e}, pixels above 1e-5: {(d > 1e-5).sum()}")
    assert np.mean(d > 1e-5) <= 1e-3 and d.max() <= 1e-2 + 1e-5
    assert po.device_errors() == 0


@pytest.mark.parametrize("kind", ["f16", "sg"])
def test_split_forms(po, fog, kind):
    s, _, _ = fog
    if kind == "sg":
        s = dict(s, lobes=scenes.sg_lobes(4, 41))
        tree = po.Tree.from_scene(s)
    else:
        tree = po.Tree.from_scene(s, dtype="f16")
    cam, pose = _cam(po, 300, 240, seed=9)
    _say(f"split render, {kind} tree")
    img = po.render_camera(tree, cam, stop_T=1e-4).cpu().numpy()
    one, _ = _one_pass(po, tree, cam, 1e-4)
    d = np.abs(img - one).max(-1)
    _say(f"{kind}: split vs one pass max {d.max():.2e}")
    assert np.mean(d > 1e-5) <= 1e-4 and d.max() <= 1e-4 + 1e-5
    sig, sh = tree.leaf_values()
    ot = oracle.OracleTree(s["depth"], s["sh_degree"], s["center"], s["half"], s["cells"], sig, sh,
                           lobes=s.get("lobes"))
    rng = np.random.default_rng(11)
    idx = rng.choice(300 * 240, 1500, replace=False)
    ref, _ = _oracle_pixels(ot, cam, pose, idx, 1e-4)
    err = np.abs(img.reshape(-1, 3)[idx] - ref).max(1)
    _say(f"{kind}: split vs oracle max {err.max():.2e}")
    assert err.max() <= TOL
    assert po.device_errors() == 0


def test_split_queue_overflow(po, fog):
    # 2048 x 2048 rays, most of them long: far more chunks than the queue
    # holds, so many rays finish their walk in the first kernel
    s, tree, ot = fog
    W = H = 2048
    cam, pose = _cam(po, W, H, seed=13, radius=2.2)
    _say(f"split render {W}x{H} (queue overflow)")
    img = po.render_camera(tree, cam, stop_T=1e-4).cpu().numpy()
    one, _ = _one_pass(po, tree, cam, 1e-4)
    d = np.abs(img - one).max(-1).reshape(-1)
    _say(f"overflow: split vs one pass max {d.max():.2e}, pixels above 1e-5: {(d > 1e-5).sum()}")
    assert np.mean(d > 1e-5) <= 1e-4 and d.max() <= 1e-4 + 1e-5
    rng = np.random.default_rng(19)
    idx = rng.choice(W * H, 2000, replace=False)
    ref, _ = _oracle_pixels(ot, cam, pose, idx, 1e-4)
    err = np.abs(img.reshape(-1, 3)[idx] - ref).max(1)
    _say(f"overflow: split vs oracle max {err.max():.2e}")
    assert err.max() <= TOL
    assert po.device_errors() == 0


def test_split_repeated_and_small(po, fog):
    # repeated frames reuse the queue; a small image below the split size in
    # between renders in one pass, identical to the batch path
    import torch

    s, tree, ot = fog
    cam, _ = _cam(po, 256, 256, seed=3)
    a = po.render_camera(tree, cam, stop_T=1e-4)
    small, _ = _cam(po, 64, 48, seed=3)
    sm = po.render_camera(tree, small, stop_T=1e-4).cpu().numpy()
    one, _ = _one_pass(po, tree, small, 1e-4)
    assert np.array_equal(sm, one)
    for _ in range(3):
        b = po.render_camera(tree, cam, stop_T=1e-4)
        torch.cuda.synchronize()
        assert torch.equal(a, b)
    # the queues can be released; the next split render makes new ones
    po.release_queues()
    b = po.render_camera(tree, cam, stop_T=1e-4)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    # a second stream gets its own queue
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        c = po.render_camera(tree, cam, stop_T=1e-4, stream=st)
    st.synchronize()
    assert torch.equal(a, c)
    assert po.device_errors() == 0


def test_reserve_queues(po, fog):
    # po_reserve_queues allocates a stream's queue up front (~201 MB); a
    # split render on that stream then allocates nothing, and a second
    # reservation of the same stream does nothing
    import torch

    s, tree, ot = fog
    po.release_queues()
    st = torch.cuda.Stream()
    cam, _ = _cam(po, 256, 256, seed=3)
    out = torch.empty((256, 256, 3), device="cuda")
    ref = po.render_camera(tree, cam, stop_T=1e-4)  # the default stream's own queue
    torch.cuda.synchronize()
    f0, _ = torch.cuda.mem_get_info()
    po.reserve_queues(stream=st)
    torch.cuda.synchronize()
    f1, _ = torch.cuda.mem_get_info()
    _say(f"reserve: {(f0 - f1) / 1e6:.1f} MB")
    assert f0 - f1 >= 190e6
    with torch.cuda.stream(st):
        po.render_camera(tree, cam, stop_T=1e-4, out=out, stream=st)
        po.reserve_queues(stream=st)
    st.synchronize()
    f2, _ = torch.cuda.mem_get_info()
    assert abs(f2 - f1) < 16e6
    assert torch.equal(out, ref)
    po.release_queues()
    torch.cuda.synchronize()
    f3, _ = torch.cuda.mem_get_info()
    assert f3 - f2 >= 380e6  # both queues freed
    assert po.device_errors() == 0


def test_split_passes_share_the_queue(po, fog):
    # every kind of split pass, one after another on one stream's queue,
    # against the same pass run alone on a fresh queue (colours bit for bit;
    # gradients within the reordering of their float atomics)
    import torch

    s, tree, ot = fog
    cam, _ = _cam(po, 256, 256, seed=5)
    cam2, _ = _cam(po, 320, 256, seed=6)
    o, d = scenes.random_rays(70000, 91, radius=2.5, spread=0.9)
    og, dg = (torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (o, d))
    gg = torch.from_numpy(np.random.default_rng(93).standard_normal((len(o), 3)).astype(np.float32)).cuda()

    def camera():
        return po.render_camera(tree, cam, stop_T=1e-4)

    def rays():
        return po.render_rays(tree, og, dg, stop_T=1e-4)

    def batch():
        a = torch.empty((256, 256, 3), device="cuda")
        b = torch.empty((256, 320, 3), device="cuda")
        po.render_batch([po.Job(tree, cam, a), po.Job(tree, cam2, b)])
        return torch.cat([a.reshape(-1), b.reshape(-1)])

    def keep_and_backward():
        slot = torch.empty(len(o), dtype=torch.int32, device="cuda")
        rk = po.render_rays_keep(tree, og, dg, slot, stop_T=1e-4)
        ks = torch.zeros((tree.n_leaves,), device="cuda")
        ksh = torch.zeros((tree.n_leaves, tree.stride), device="cuda")
        po.render_rays_backward_kept(tree, og, dg, rk, gg, slot, ks, ksh, stop_T=1e-4)
        return rk, ks, ksh

    def backward():
        gs, gsh = po.render_rays_backward(tree, og, dg, rays(), gg, stop_T=1e-4)
        return gs, gsh

    passes = [("camera", camera), ("rays", rays), ("batch", batch), ("keep", keep_and_backward),
              ("backward", backward), ("camera again", camera), ("keep again", keep_and_backward)]
    alone = {}
    for name, f in passes:
        po.release_queues()
        alone[name] = f()
        torch.cuda.synchronize()
    po.release_queues()
    _say("split passes in a row on one queue")
    for rnd in range(2):
        for name, f in passes:
            got = f()
            torch.cuda.synchronize()
            want = alone[name]
            if not isinstance(got, tuple):
                assert torch.equal(got, want), f"{name} (round {rnd})"
                continue
            for i, (x, y) in enumerate(zip(got, want)):
                if x.shape[-1] == 3 and x.dim() == 2 and x.shape[0] == len(o):
                    assert torch.equal(x, y), f"{name} colours (round {rnd})"
                else:
                    scale = float(y.abs().max())
                    assert float((x - y).abs().max()) <= 1e-5 * scale, f"{name} output {i} (round {rnd})"
    assert po.device_errors() == 0


@pytest.mark.parametrize("deg,sg,dtype", [(0, False, "f32"), (1, False, "f16"), (2, False, "f32"), (4, False, "f32"),
                                          (4, True, "f16")])
def test_split_every_basis(po, deg, sg, dtype):
    # every compiled K (1, 4, 9, 25) and SG-25 through the split render, on
    # the depth-7 blob band at 320 x 256 pixels
    s = scenes.scene_blobs(depth=7, sh_degree=deg, seed=6, data_seed=7)
    K = (deg + 1) ** 2
    if sg:
        s = dict(s, lobes=scenes.sg_lobes(K, 43))
    tree = po.Tree.from_scene(s, dtype=dtype)
    cam, pose = _cam(po, 320, 256, seed=21, radius=3.0)
    _say(f"split render K={K} sg={sg} {dtype}")
    img = po.render_camera(tree, cam, stop_T=1e-4).cpu().numpy()
    one, aux = _one_pass(po, tree, cam, 1e-4, aux=True)
    assert (aux[..., 2] > 32).sum() > 500  # walks long enough to be split
    d = np.abs(img - one).max(-1)
    assert np.mean(d > 1e-5) <= 1e-4 and d.max() <= 1e-4 + 1e-5
    sig, sh = tree.leaf_values()
    ot = oracle.OracleTree(s["depth"], deg, s["center"], s["half"], s["cells"], sig, sh, lobes=s.get("lobes"))
    rng = np.random.default_rng(23)
    idx = np.unique(np.concatenate([rng.choice(320 * 256, 1200, replace=False),
                                    np.argsort(-aux[..., 2].reshape(-1))[:200]]))
    ref, _ = _oracle_pixels(ot, cam, pose, idx, 1e-4)
    err = np.abs(img.reshape(-1, 3)[idx] - ref).max(1)
    _say(f"K={K} sg={sg} {dtype}: split vs oracle max {err.max():.2e}")
    assert err.max() <= TOL
    assert po.device_errors() == 0


def test_split_max_depth(po):
    # the deepest tree the ABI accepts (depth 15): a dense cluster of finest
    # cells plus coarse leaves, seen by a 256 x 256 camera close to the cluster
    from paper_2103_14024_amd import _lib as L

    depth = L.PO_MAX_DEPTH
    base = (1 << depth) // 2 - 12
    g = np.stack(np.meshgrid(*[np.arange(24)] * 3, indexing="ij"), -1).reshape(-1, 3) + base
    fine = np.column_stack([np.full(len(g), depth), g])
    coarse = np.array([[3, 0, 0, 0], [3, 7, 7, 7], [2, 0, 3, 1], [4, 15, 2, 9]])
    cells = np.concatenate([fine, coarse]).astype(np.int32)
    sigma, sh = scenes.leaf_values(len(cells), 1, 16, mu=7.0, s=0.3)
    s = dict(depth=depth, sh_degree=1, center=(0.0, 0.0, 0.0), half=1.0, cells=cells, sigma=sigma, sh=sh)
    tree = po.Tree.from_scene(s)
    cell = 2.0 / (1 << depth)
    pose = scenes.look_at(np.array([0.3, -0.2, 0.25]) * 24 * cell * 3, (0.0, 0.0, 0.0))
    fx, fy, cx, cy = scenes.intrinsics(256, 256, 60.0)
    cam = po.Camera(pose, 256, 256, fx, fy, cx, cy)
    _say("split render, depth-15 tree")
    img = po.render_camera(tree, cam, stop_T=1e-4).cpu().numpy()
    one, aux = _one_pass(po, tree, cam, 1e-4, aux=True)
    _say(f"depth 15: max steps {aux[..., 2].max():.0f}, rays past 32 cells {(aux[..., 2] > 32).sum()}")
    assert (aux[..., 2] > 32).sum() > 2000
    d = np.abs(img - one).max(-1)
    assert np.mean(d > 1e-5) <= 1e-4 and d.max() <= 1e-4 + 1e-5
    ot = oracle.OracleTree(depth, 1, s["center"], s["half"], cells, sigma, sh)
    rng = np.random.default_rng(29)
    idx = np.unique(np.concatenate([rng.choice(256 * 256, 1500, replace=False),
                                    np.argsort(-aux[..., 2].reshape(-1))[:200]]))
    ref, _ = _oracle_pixels(ot, cam, pose, idx, 1e-4)
    err = np.abs(img.reshape(-1, 3)[idx] - ref).max(1)
    _say(f"depth 15: split vs oracle max {err.max():.2e}")
    assert err.max() <= TOL
    assert po.device_errors() == 0


@pytest.mark.parametrize("stop_T", [0.0, 1e-4])
def test_split_ray_list(po, fog, stop_T):
    # ray-list renders of >= 65536 rays are split too (pieces of 8 cells
    # below 2^18 rays, as in a camera render above); the one-pass reference
    # renders the list in runs of 65535 rays
    import torch

    s, tree, ot = fog
    cam, pose = _cam(po, 512, 512, seed=3)
    f32 = [float(np.float32(v)) for v in (cam.fx, cam.fy, cam.cx, cam.cy)]
    o, d = oracle.camera_rays(np.asarray(pose, np.float32).astype(np.float64), 512, 512, *f32)
    o2, d2 = scenes.random_rays(20000, 37, radius=2.5, spread=0.9)
    o = np.concatenate([o, o2]).astype(np.float32)
    d = np.concatenate([d, d2]).astype(np.float32)
    n = len(o)
    _say(f"split ray list, {n} rays, stop_T {stop_T}")
    og, dg = torch.from_numpy(o).cuda(), torch.from_numpy(d).cuda()
    rgb = po.render_rays(tree, og, dg, stop_T=stop_T).cpu().numpy()
    runs = [po.render_rays(tree, og[a:a + 65535], dg[a:a + 65535], stop_T=stop_T, aux=True)
            for a in range(0, n, 65535)]
    one = np.concatenate([r[0].cpu().numpy() for r in runs])
    aux = np.concatenate([r[1].cpu().numpy() for r in runs])
    assert (aux[:, 2] > 32).sum() > 60000
    dd = np.abs(rgb - one).max(1)
    _say(f"ray list: split vs one pass max {dd.max():.2e}, above 1e-5: {(dd > 1e-5).sum()}")
    assert np.mean(dd > 1e-5) <= 1e-4 and dd.max() <= stop_T + 1e-5
    # one ray fewer than the split size renders in one pass, bit-identical
    small = po.render_rays(tree, og[:65535], dg[:65535], stop_T=stop_T).cpu().numpy()
    assert np.array_equal(small, one[:65535])
    # a list just above it is split with small pieces
    mid = po.render_rays(tree, og[:70000], dg[:70000], stop_T=stop_T).cpu().numpy()
    dm = np.abs(mid - one[:70000]).max(1)
    assert np.mean(dm > 1e-5) <= 1e-4 and dm.max() <= stop_T + 1e-5
    rng = np.random.default_rng(31)
    idx = np.unique(np.concatenate([rng.choice(n, 2000, replace=False), np.argsort(-aux[:, 2])[:300]]))
    ref, _, _, _ = ot.render_rays(o[idx].astype(np.float64), d[idx].astype(np.float64), gamma=stop_T)
    err = np.abs(rgb[idx] - ref).max(1)
    _say(f"ray list: split vs oracle max {err.max():.2e}")
    assert err.max() <= TOL
    assert po.device_errors() == 0


def test_split_codebook(po, fog):
    # codebook leaves (App. B.2) through the split render: the oracle renders
    # the leaves its own codebooks decode to
    s, _, _ = fog
    M = 256
    tree = po.Tree.from_cells_codebook(s["depth"], s["sh_degree"], s["cells"], s["sigma"], s["sh"], M, s["center"],
                                       s["half"])
    cam, pose = _cam(po, 288, 256, seed=17)
    _say("split render, codebook tree")
    img = po.render_camera(tree, cam, stop_T=1e-4).cpu().numpy()
    one, _ = _one_pass(po, tree, cam, 1e-4)
    d = np.abs(img - one).max(-1)
    _say(f"codebook: split vs one pass max {d.max():.2e}")
    assert np.mean(d > 1e-5) <= 1e-4 and d.max() <= 1e-4 + 1e-5
    idx_, books = oracle.codebook(np.asarray(s["sh"], np.float32), M)
    sig16 = np.asarray(s["sigma"], np.float32).astype(np.float16).astype(np.float64)
    ot = oracle.OracleTree(s["depth"], s["sh_degree"], s["center"], s["half"], s["cells"], sig16,
                           oracle.codebook_decode(idx_, books))
    rng = np.random.default_rng(37)
    idx = rng.choice(288 * 256, 1500, replace=False)
    ref, _ = _oracle_pixels(ot, cam, pose, idx, 1e-4)
    err = np.abs(img.reshape(-1, 3)[idx] - ref).max(1)
    _say(f"codebook: split vs oracle max {err.max():.2e}")
    assert err.max() <= TOL
    assert po.device_errors() == 0


@pytest.mark.parametrize("scene,gamma", [("fog", 1e-4), ("fog", 1e-2), ("blobs", 1e-4), ("blobs", 0.0),
                                         ("blobs", 1e-2)])
def test_split_backward(po, fog, scene, gamma):
    # backward passes of >= 65536 rays run in pieces; the split gradient and
    # the one-pass gradient (two halves of 35000 rays) are each held to the
    # FP64 oracle gradient under the threshold-straddle rule
    import torch

    if scene == "fog":
        s, tree, ot = fog
        o, d = scenes.random_rays(70000, 41, radius=2.5, spread=0.9)
    else:
        s = scenes.scene_blobs(depth=7, sh_degree=2, seed=8, data_seed=9)
        tree = po.Tree.from_scene(s)
        ot = oracle.OracleTree(s["depth"], s["sh_degree"], s["center"], s["half"], s["cells"], s["sigma"], s["sh"])
        o, d = scenes.random_rays(70000, 43, radius=2.0, spread=0.8)
    _say(f"split backward, {scene}, stop_T {gamma}")
    g = np.random.default_rng(47).standard_normal((len(o), 3)).astype(np.float32)
    bg = (0.9, 0.4, 0.1)
    og, dg, gg = (torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (o, d, g))
    # each backward differentiates the colour of the render that cuts the rays
    # alike (the same float transmittances, so the same early stop): the
    # split render for the split backward, the one-pass render for the halves
    rgb = po.render_rays(tree, og, dg, bg=bg, stop_T=gamma)
    rgb1 = po.render_rays(tree, og, dg, bg=bg, stop_T=gamma, one_pass=True)
    gs, gsh = po.render_rays_backward(tree, og, dg, rgb, gg, bg=bg, stop_T=gamma)
    h = len(o) // 2
    hs = torch.zeros_like(gs)
    hsh = torch.zeros_like(gsh)
    for a, b in ((0, h), (h, len(o))):
        po.render_rays_backward(tree, og[a:b], dg[a:b], rgb1[a:b], gg[a:b], bg=bg, stop_T=gamma, grad_sigma=hs,
                                grad_sh=hsh)
    # the kept render and the backward over its own pieces
    slot = torch.empty(len(o), dtype=torch.int32, device="cuda")
    rgbk = po.render_rays_keep(tree, og, dg, slot, bg=bg, stop_T=gamma)
    ks, ksh = torch.zeros_like(gs), torch.zeros_like(gsh)
    po.render_rays_backward_kept(tree, og, dg, rgbk, gg, slot, ks, ksh, bg=bg, stop_T=gamma)
    torch.cuda.synchronize()
    assert float((rgbk - rgb).abs().max()) <= 1e-6
    assert int((slot >= 0).sum()) > 0
    (ls, hs_), (lh, hh), n_str = gradcheck.grad_envelope(ot, o, d, g, bg, gamma)
    _say(f"{scene} {gamma}: {n_str} of {len(o)} rays straddle stop_T")
    for path, (x, y) in (("split", (gs, gsh)), ("one pass", (hs, hsh)), ("kept", (ks, ksh))):
        a, b = gradcheck.to_cells(tree, x.cpu().numpy(), y.cpu().numpy())
        gradcheck.check(a, ls, hs_, f"{scene} {gamma} {path} dsigma")
        gradcheck.check(b, lh, hh, f"{scene} {gamma} {path} dsh")
    assert po.device_errors() == 0


def test_split_backward_training_shape(po):
    # the differentiation workload's shape: the depth-8 blob band (SH degree
    # 2), a random batch of 65536 pixels of 400x400 views, a perturbed copy
    # rendered against the ground truth; upstream gradient of the mean squared
    # error, as one optimisation step computes it
    import torch

    gt = scenes.scene_train()
    sig, sh = scenes.perturb(gt["sigma"], gt["sh"], 0.3, 7)
    _say(f"split backward, training shape: {len(gt['cells'])} leaves, 65536 rays")
    tree = po.Tree.from_cells(gt["depth"], gt["sh_degree"], gt["cells"], sig, sh)
    gt_tree = po.Tree.from_scene(gt)
    W = H = 400
    fx, fy, cx, cy = scenes.intrinsics(W, H, 40.0)
    poses = scenes.hemisphere_poses(100, 4.0, 5)
    rng = np.random.default_rng(11)
    pick = rng.integers(0, 8, 65536)
    pix = rng.integers(0, W * H, 65536)
    f32 = [float(np.float32(v)) for v in (fx, fy, cx, cy)]
    o = np.empty((65536, 3), np.float32)
    d = np.empty((65536, 3), np.float32)
    for k in range(8):
        ok, dk = oracle.camera_rays(np.asarray(poses[k], np.float32).astype(np.float64), W, H, *f32)
        m = pick == k
        o[m] = ok[pix[m]]
        d[m] = dk[pix[m]]
    og, dg = torch.from_numpy(o).cuda(), torch.from_numpy(d).cuda()
    target = po.render_rays(gt_tree, og, dg, stop_T=1e-4)
    rgb = po.render_rays(tree, og, dg, stop_T=1e-4)
    gg = (2.0 / rgb.numel()) * (rgb - target)
    gs, gsh = po.render_rays_backward(tree, og, dg, rgb, gg.contiguous(), stop_T=1e-4)
    # the training step's path: the kept render and the backward over its pieces
    slot = torch.empty(65536, dtype=torch.int32, device="cuda")
    rgbk = po.render_rays_keep(tree, og, dg, slot, stop_T=1e-4)
    ks, ksh = torch.zeros_like(gs), torch.zeros_like(gsh)
    po.render_rays_backward_kept(tree, og, dg, rgbk, gg.contiguous(), slot, ks, ksh, stop_T=1e-4)
    torch.cuda.synchronize()
    assert float((rgbk - rgb).abs().max()) <= 1e-6
    g = gg.cpu().numpy().astype(np.float64)
    ot = oracle.OracleTree(gt["depth"], gt["sh_degree"], gt["center"], gt["half"], gt["cells"], sig, sh)
    (ls, hs_), (lh, hh), n_str = gradcheck.grad_envelope(ot, o, d, g, (1.0, 1.0, 1.0), 1e-4)
    _say(f"training shape: {n_str} straddling rays")
    for path, (x, y) in (("split", (gs, gsh)), ("kept", (ks, ksh))):
        a, b = gradcheck.to_cells(tree, x.cpu().numpy(), y.cpu().numpy())
        gradcheck.check(a, ls, hs_, f"training shape {path} dsigma")
        gradcheck.check(b, lh, hh, f"training shape {path} dsh")
    assert po.device_errors() == 0


@pytest.mark.parametrize("deg", [1, 4])
def test_kept_backward_sg(po, deg):
    # the kept render and its backward over spherical-Gaussian leaves (K = 4
    # and 25) against the FP64 oracle gradient, 70000 rays of the depth-6
    # blob band (the render splits them)
    import torch

    K = (deg + 1) ** 2
    s = scenes.scene_blobs(depth=6, sh_degree=deg, seed=12, data_seed=13)
    s = dict(s, lobes=scenes.sg_lobes(K, 47))
    tree = po.Tree.from_scene(s)
    ot = oracle.OracleTree(s["depth"], deg, s["center"], s["half"], s["cells"], s["sigma"], s["sh"], lobes=s["lobes"])
    o, d = scenes.random_rays(70000, 59, radius=2.0, spread=0.8)
    g = np.random.default_rng(61).standard_normal((len(o), 3)).astype(np.float32)
    og, dg, gg = (torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (o, d, g))
    _say(f"kept backward, SG K={K}")
    slot = torch.empty(len(o), dtype=torch.int32, device="cuda")
    rgb = po.render_rays_keep(tree, og, dg, slot, stop_T=1e-4)
    ks = torch.zeros((tree.n_leaves,), device="cuda")
    ksh = torch.zeros((tree.n_leaves, tree.stride), device="cuda")
    po.render_rays_backward_kept(tree, og, dg, rgb, gg, slot, ks, ksh, stop_T=1e-4)
    torch.cuda.synchronize()
    assert int((slot >= 0).sum()) > 1000
    (ls, hs_), (lh, hh), n_str = gradcheck.grad_envelope(ot, o, d, g, (1.0, 1.0, 1.0), 1e-4)
    a, b = gradcheck.to_cells(tree, ks.cpu().numpy(), ksh.cpu().numpy())
    gradcheck.check(a, ls, hs_, f"SG K={K} kept dsigma")
    gradcheck.check(b, lh, hh, f"SG K={K} kept dsh")
    assert po.device_errors() == 0


@pytest.mark.parametrize("between", [False, True])
def test_autograd_split(po, fog, between):
    # the autograd function over 70000 rays (split render): its backward
    # differentiates over the kept pieces, or, after another split render on
    # the stream, walks the rays again; either is held to the oracle gradient
    import torch

    s, tree, ot = fog
    tree.sigma.requires_grad_(True)
    tree.sh.requires_grad_(True)
    try:
        o, d = scenes.random_rays(70000, 67, radius=2.5, spread=0.9)
        og, dg = (torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (o, d))
        g = np.random.default_rng(71).standard_normal((len(o), 3)).astype(np.float32)
        rgb = po.render_rays_differentiable(tree, og, dg, stop_T=1e-4)
        if between:
            po.render_rays(tree, og, dg)  # other split work on the stream's queue
        rgb.backward(torch.from_numpy(g).cuda())
        torch.cuda.synchronize()
        (ls, hs_), (lh, hh), n_str = gradcheck.grad_envelope(ot, o, d, g, (1.0, 1.0, 1.0), 1e-4)
        a, b = gradcheck.to_cells(tree, tree.sigma.grad.cpu().numpy(), tree.sh.grad.cpu().numpy())
        gradcheck.check(a, ls, hs_, f"autograd (between {between}) dsigma")
        gradcheck.check(b, lh, hh, f"autograd (between {between}) dsh")
    finally:
        tree.sigma.requires_grad_(False)
        tree.sh.requires_grad_(False)
        tree.sigma.grad = None
        tree.sh.grad = None
    assert po.device_errors() == 0


def test_kept_backward_refusals(po, fog):
    # the backward over kept pieces runs only right after the kept render of
    # the same rays and options on the same stream, and only once
    import torch

    from paper_2103_14024_amd._lib import PlenOctreeError

    s, tree, ot = fog
    o, d = scenes.random_rays(70000, 53, radius=2.5, spread=0.9)
    og, dg = (torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (o, d))
    gg = torch.full((len(o), 3), 1e-3, device="cuda")
    slot = torch.empty(len(o), dtype=torch.int32, device="cuda")
    gs = torch.zeros((tree.n_leaves,), device="cuda")
    gsh = torch.zeros((tree.n_leaves, tree.stride), device="cuda")
    rgb = po.render_rays_keep(tree, og, dg, slot)
    po.render_rays(tree, og, dg)  # a split render on the same stream's queue
    with pytest.raises(PlenOctreeError):
        po.render_rays_backward_kept(tree, og, dg, rgb, gg, slot, gs, gsh)
    rgb = po.render_rays_keep(tree, og, dg, slot)
    with pytest.raises(PlenOctreeError):
        po.render_rays_backward_kept(tree, og, dg, rgb, gg, slot, gs, gsh, stop_T=1e-2)
    po.render_rays_backward_kept(tree, og, dg, rgb, gg, slot, gs, gsh)
    with pytest.raises(PlenOctreeError):
        po.render_rays_backward_kept(tree, og, dg, rgb, gg, slot, gs, gsh)  # consumed
    with pytest.raises(ValueError):
        po.render_rays_keep(tree, og, dg, slot[:100])
    # below 65536 rays both run in one pass: the same gradient as the plain backward
    n = 5000
    rgb_s = po.render_rays_keep(tree, og[:n], dg[:n], slot[:n])
    ks, ksh = torch.zeros_like(gs), torch.zeros_like(gsh)
    po.render_rays_backward_kept(tree, og[:n], dg[:n], rgb_s, gg[:n], slot[:n], ks, ksh)
    ps, psh = po.render_rays_backward(tree, og[:n], dg[:n], rgb_s, gg[:n])
    torch.cuda.synchronize()
    assert torch.allclose(ks, ps, rtol=1e-5, atol=1e-9) and torch.allclose(ksh, psh, rtol=1e-5, atol=1e-9)
    assert po.device_errors() == 0


@pytest.mark.parametrize("kind", ["aux", "sh_off", "clip"])
def test_split_view(po, fog, kind):
    # the viewer variant through the split render: depth integral, samples
    # and cells composed over the pieces, against the one-pass batch render
    # and the oracle
    import torch

    s, tree, ot = fog
    W = H = 256
    cam, pose = _cam(po, W, H, seed=3)
    off, plane = 0, None
    if kind == "sh_off":
        off = 0b0110
    if kind == "clip":
        plane = (0.3, -0.2, 0.9, 0.1)
    _say(f"split viewer render: {kind}")
    img, aux = po.render_camera(tree, cam, stop_T=1e-4, aux=True, sh_off=off, clip=plane)
    img, aux = img.cpu().numpy().reshape(-1, 3), aux.cpu().numpy().reshape(-1, 4)
    out = torch.empty((H, W, 3), device="cuda")
    a1 = torch.empty((H, W, 4), device="cuda")
    po.render_batch([po.Job(tree, cam, out, stop_T=1e-4, aux_out=a1, sh_off=off, clip=plane, one_pass=True)])
    torch.cuda.synchronize()
    one, a1 = out.cpu().numpy().reshape(-1, 3), a1.cpu().numpy().reshape(-1, 4)
    assert (a1[:, 2] > 32).sum() > 10000
    d = np.abs(img - one).max(1)
    _say(f"{kind}: rgb vs one pass max {d.max():.2e}; T {np.abs(aux[:, 0] - a1[:, 0]).max():.2e}; "
         f"depth {np.abs(aux[:, 3] - a1[:, 3]).max():.2e}; samples equal {np.mean(aux[:, 1] == a1[:, 1]):.4f}; "
         f"cells equal {np.mean(aux[:, 2] == a1[:, 2]):.4f}, max diff {np.abs(aux[:, 2] - a1[:, 2]).max():.0f}, "
         f"mean split - one pass {np.mean(aux[:, 2] - a1[:, 2]):.3f}")
    assert np.mean(d > 1e-5) <= 1e-4 and d.max() <= 1e-4 + 1e-5
    assert np.abs(aux[:, 0] - a1[:, 0]).max() <= 1e-4 + 1e-5
    assert np.abs(aux[:, 3] - a1[:, 3]).max() <= 1e-4 * (np.abs(a1[:, 3]).max() + 1.0)
    # samples: a cell cut between two pieces counts once
    assert np.mean(aux[:, 1] == a1[:, 1]) > 0.99 and np.abs(aux[:, 1] - a1[:, 1]).max() <= 2
    # cells: a piece that starts on a face can visit the cell behind it for zero length
    assert np.mean(aux[:, 2] == a1[:, 2]) > 0.9 and np.abs(aux[:, 2] - a1[:, 2]).max() <= 4
    f32 = [float(np.float32(v)) for v in (cam.fx, cam.fy, cam.cx, cam.cy)]
    o, dd = oracle.camera_rays(np.asarray(pose, np.float32).astype(np.float64), W, H, *f32)
    rng = np.random.default_rng(53)
    idx = np.unique(np.concatenate([rng.choice(W * H, 1500, replace=False), np.argsort(-a1[:, 2])[:200]]))
    rr, T, ns, dep = ot.render_view(o[idx], dd[idx], gamma=1e-4, sh_off=off,
                                    clip=None if plane is None else np.asarray(plane, np.float32))
    _say(f"{kind}: vs oracle rgb {np.abs(img[idx] - rr).max():.2e} T {np.abs(aux[idx, 0] - T).max():.2e} "
         f"depth {np.abs(aux[idx, 3] - dep).max():.2e}")
    assert np.abs(img[idx] - rr).max() <= TOL
    assert np.abs(aux[idx, 0] - T).max() <= TOL
    assert np.all(np.abs(aux[idx, 3] - dep) <= TOL * (np.linalg.norm(o[idx], axis=1) + 2 * np.sqrt(3.0)))
    assert np.mean(aux[idx, 1] == ns) > 0.99 and np.abs(aux[idx, 1] - ns).max() <= 2
    assert po.device_errors() == 0
