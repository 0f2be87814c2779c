"""Host-side logic of the render server (no GPU): the output arena's
first-fit allocation and coalescing, and the request generator."""
import numpy as np

from paper_2103_14024_amd import server


class _FakeArena(server.Arena):
    def __init__(self, n):
        self.size, self.free, self.used = n, [(0, n)], 0


def test_arena_first_fit_and_merge():
    a = _FakeArena(4096)
    x = a.alloc(1000)   # -> 1024 bytes
    y = a.alloc(1000)
    z = a.alloc(2048)
    assert (x, y, z) == (0, 1024, 2048) and a.used == 4096
    assert a.alloc(1) == -1
    a.release(y, 1000)
    assert a.alloc(2000) == -1          # only 1024 free
    a.release(x, 1000)
    assert a.free == [(0, 2048)]        # neighbours merged
    assert a.alloc(2000) == 0
    a.release(0, 2000)
    a.release(z, 2048)
    assert a.free == [(0, 4096)] and a.used == 0


def test_poisson_requests():
    reqs = server.poisson_requests(4000, 200.0, 4, seed=3)
    arr = np.array([r.arrival for r in reqs])
    assert np.all(np.diff(arr) > 0)
    rate = len(arr) / arr[-1]
    assert 180 < rate < 220
    res = {(r.cam.width, r.cam.height) for r in reqs}
    assert res == set(server.RESOLUTIONS)
    assert {r.scene for r in reqs} == {0, 1, 2, 3}
    # cameras on the upper hemisphere, radius 4
    pos = np.array([np.asarray(r.cam.c2w)[:, 3] for r in reqs[:200]])
    assert np.all(pos[:, 2] >= 0) and np.allclose(np.linalg.norm(pos, axis=1), 4.0, atol=1e-5)
    again = server.poisson_requests(4000, 200.0, 4, seed=3)
    assert [r.arrival for r in again] == list(arr)
