"""Tree checkpoints (.npz of plain arrays, read without unpickling): round
trips of every leaf form, and the host-side checks that refuse malformed or
pickled files before anything reaches a device.  Host only."""
import numpy as np
import pytest

from paper_2103_14024_amd import _lib as L
from paper_2103_14024_amd import scenes
from paper_2103_14024_amd.tree import build_host, default_stride, read_checkpoint, write_checkpoint


def _fields(dtype=np.float32, sg=False):
    sc = scenes.scene_small()
    child, perm = build_host(sc["depth"], sc["sh_degree"], sc["cells"], sc["center"], sc["half"])
    n, K = len(perm), scenes.n_coef(sc["sh_degree"])
    rec = np.zeros((n, default_stride(sc["sh_degree"])), dtype)
    rec[:, :3 * K] = np.asarray(sc["sh"], np.float32).reshape(n, 3 * K)[perm]
    f = {"depth": sc["depth"], "sh_degree": sc["sh_degree"], "center": sc["center"], "half": sc["half"],
         "child": child, "sigma": np.asarray(sc["sigma"], np.float32)[perm].astype(dtype), "sh": rec, "perm": perm}
    if sg:
        f["lobes"] = scenes.sg_lobes(K, 17).astype(np.float32)
    return f


@pytest.mark.parametrize("dtype,sg", [(np.float32, False), (np.float16, False), (np.float32, True)])
def test_round_trip(tmp_path, dtype, sg):
    f = _fields(dtype, sg)
    p = tmp_path / "t.npz"
    write_checkpoint(p, f, {"step": 123, "seed": 7, "rng": np.arange(16, dtype=np.uint8)})
    g, meta = read_checkpoint(p)
    for k in ("child", "sigma", "sh", "perm") + (("lobes",) if sg else ()):
        assert g[k].dtype == f[k].dtype and np.array_equal(g[k], f[k]), k
    assert (g["depth"], g["sh_degree"], g["half"]) == (f["depth"], f["sh_degree"], f["half"])
    assert g["center"] == tuple(float(c) for c in f["center"])
    assert g["codebook"] is None and (sg or g["lobes"] is None)
    assert int(meta["step"]) == 123 and int(meta["seed"]) == 7 and np.array_equal(meta["rng"], np.arange(16))


def test_codebook_round_trip(tmp_path):
    f = _fields(np.float16)
    n, K = f["sigma"].shape[0], scenes.n_coef(f["sh_degree"])
    f["sh"] = np.random.default_rng(0).integers(-32768, 32767, (n, K), dtype=np.int16)
    f["codebook"] = np.random.default_rng(1).standard_normal((K, 64, 4)).astype(np.float16)
    p = tmp_path / "cb.npz"
    write_checkpoint(p, f)
    g, meta = read_checkpoint(p)
    assert np.array_equal(g["sh"], f["sh"]) and np.array_equal(g["codebook"], f["codebook"]) and meta == {}


def test_pickled_arrays_refused(tmp_path):
    # an object array can only be stored pickled; the reader never unpickles
    f = _fields()
    p = tmp_path / "obj.npz"
    arrays = {"version": np.int32(1), "depth": np.int32(f["depth"]), "sh_degree": np.int32(f["sh_degree"]),
              "center": np.zeros(3), "half": np.float64(1.0), "child": f["child"], "sigma": f["sigma"],
              "sh": np.array([object()] * 3, dtype=object)}
    np.savez(p, **arrays)
    with pytest.raises(ValueError):
        read_checkpoint(p)


def test_malformed_refused(tmp_path):
    f = _fields()
    cases = {
        "child dtype": dict(child=f["child"].astype(np.int64)),
        "leaf count": dict(sigma=f["sigma"][:-1]),
        "record width": dict(sh=f["sh"][:, :5]),
        "mixed dtypes": dict(sh=f["sh"].astype(np.float16)),
        "perm length": dict(perm=f["perm"][:-1]),
    }
    for name, change in cases.items():
        g = dict(f, **change)
        p = tmp_path / "bad.npz"
        write_checkpoint(p, g)
        with pytest.raises(ValueError):
            read_checkpoint(p)
    # a child entry past the leaf count: caught by the library's validator
    bad = f["child"].copy()
    bad[bad < 0] = np.int32(-len(f["perm"]) - 5)
    write_checkpoint(tmp_path / "bad.npz", dict(f, child=bad))
    with pytest.raises(L.PlenOctreeError):
        read_checkpoint(tmp_path / "bad.npz")
    with pytest.raises(TypeError):
        write_checkpoint(tmp_path / "m.npz", f, {"name": "text"})
