"""Sizes past 32-bit element offsets.  A lattice beyond 2^31 population elements
and taller than a grid's 65535-row extent: 4096 x 70000 FP64 (2.58e9 elements,
20.6 GB per buffer); windows around nodes near the first and the last rows, where
the element offsets pass 2^31, are stepped by the oracle from the same initial
state and compared with the device densities after each tile family (three, two
and one steps per launch).  A batch whose last run starts past element 2^31 of
its pool, against a single lattice."""
import numpy as np
import pytest

from oracle import lbm as olbm
from tests.gpu_common import CS, mirror_tile, pair, slab_rho

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import torch
    from paper_1204_4098_amd import lbm
    assert torch.cuda.is_available()
    lbm.lib()
    return lbm


def test_lattice_beyond_2_31_elements(L):
    nx, ny, half = 4096, 70000, 20
    assert 9 * nx * ny > 2 ** 31 and ny > 65535
    gp, op = pair(L, nx, ny, t=0.8, tau=0.8, scheme=2, sigma=0.1)
    rho0 = slab_rho(nx, ny, CS, 0.8, seed=51)        # seeded noise: every row differs
    pts = [(0, ny - 1), (nx - 1, ny - 3), (1024, 0), (3000, 66000), (2048, 40000)]
    wins = {}
    for cx, cy in pts:
        ys = np.arange(cy - half, cy + half) % ny
        xs = np.arange(cx - half, cx + half) % nx
        wins[(cx, cy)] = mirror_tile(olbm.init_equilibrium(np.ascontiguousarray(rho0[np.ix_(ys, xs)])))
    wp = olbm.Params(**{**op.__dict__, "nx": 4 * half, "ny": 4 * half})
    lat = L.Lattice(gp, rho0)
    del rho0
    done = 0
    for tile, k in [((4, 0, 1, 3), 3), ((4, 0, 2, 2), 2), ((16, 0, 1, 1), 1)]:
        lat.set_tile(*tile)
        lat.step(k)
        done += k
        st, _, _ = lat.status()
        assert st == L.LBM_OK
        rho = lat.moments()[0]
        m = 2 * done + 1                            # light cone of `done` steps
        for cx, cy in pts:
            win = wins[(cx, cy)]
            assert olbm.step(wp, win, k)[0] == olbm.OK
            ref = olbm.moments(wp, win)[0][m:2 * half - m, m:2 * half - m]
            ys = np.arange(cy - half + m, cy + half - m) % ny
            xs = np.arange(cx - half + m, cx + half - m) % nx
            got = rho[np.ix_(ys, xs)]
            err = float(np.max(np.abs(got - ref) / ref))
            assert err < 1e-12, (tile, (cx, cy), err)
        del rho
    lat.close()


def test_batch_run_past_2_31_elements(L):
    # two 4096 x 30000 FP64 runs (1.1e9 elements each) put the third run's
    # populations past element 2^31 of the pool; that run, stepped by the batched
    # one- and two-step kernels, equals a single lattice bit for bit
    big, _ = pair(L, 4096, 30000, t=0.8, tau=0.9, scheme=2, sigma=0.1)
    small, _ = pair(L, 96, 32, t=0.8, tau=0.8, scheme=2, sigma=0.1)
    rb = slab_rho(4096, 30000, CS, 0.8, seed=61)
    rs = slab_rho(96, 32, CS, 0.8, seed=62)
    assert 2 * 9 * 4096 * 30000 > 2 ** 31
    lat = L.Lattice(small, rs)
    lat.step(7)
    want = lat.get_populations()[0].tobytes()
    lat.close()
    for tile in [(2, 0, 2, 2), (4, 8, 2, 1)]:
        b = L.Batch([big, big, small], [rb, rb, rs])
        b.set_tile(*tile)
        b.step(7)
        assert b.get_populations(2).tobytes() == want, tile
        b.close()
