"""The three-step kernel (three time steps per launch, FP64 collision
arithmetic): bitwise equal to single steps, against the FP64 oracle, through
graphs with remainders, on edge shapes and around the strip-count thresholds."""
import numpy as np
import pytest

from oracle import lbm as olbm
from tests.gpu_common import CS, PR, pair, rel_err, slab_rho

pytestmark = pytest.mark.gpu

TOL64 = 1e-10


@pytest.fixture(scope="module")
def L():
    import torch
    from paper_1204_4098_amd import lbm
    assert torch.cuda.is_available()
    lbm.lib()
    return lbm


def _run(L, gp, rho0, tile, n, graph=0):
    lat = L.Lattice(gp, rho0)
    lat.set_tile(*tile)
    if graph:
        lat.set_graph_steps(graph)
    lat.step(n)
    st, done, div = lat.status()
    f = lat.get_populations()[0]
    lat.close()
    return f, st, done, div


@pytest.mark.parametrize("precision", [0, 3])
def test_three_step_tiles_bitwise(L, precision):
    # 37 steps = 12 three-step launches and one single step; 38 ends with a
    # two-step launch
    gp, _ = pair(L, 200, 90, t=0.8, tau=0.7, scheme=2, sigma=0.1, precision=precision)
    rho0 = slab_rho(200, 90, CS, 0.8, seed=3)
    for n in (37, 38):
        ref = _run(L, gp, rho0, (2, 8, 1), n)[0]
        for tile in [(4, 0, 1, 3), (4, 64, 1, 3), (4, 5, 1, 3), (4, 1, 1, 3), (4, 128, 1, 3), (8, 0, 1, 3),
                     (8, 16, 1, 3)]:
            f, st, done, div = _run(L, gp, rho0, tile, n)
            assert st == L.LBM_OK and done == n and div == -1
            assert np.array_equal(f, ref), (n, tile)


@pytest.mark.parametrize("k", [8, 10, 12])
def test_three_step_graph_replay_bitwise(L, k):
    # graphs of k steps: k/3 three-step launches and a remainder launch of k % 3
    # steps (none for 12: 4 launches; one single step for 10: 4 launches, the
    # buffer parity unchanged per replay; a two-step launch for 8: 3 launches,
    # the parity flips per replay), an eager head and tail, against single steps
    gp, _ = pair(L, 300, 70, t=0.8, tau=0.8, scheme=2, sigma=0.105)
    rho0 = slab_rho(300, 70, CS, 0.8, seed=6)
    a = L.Lattice(gp, rho0)
    a.set_tile(2, 8, 1)
    a.step(4 + 4 * k + 5)
    fa = a.get_populations()[0]
    b = L.Lattice(gp, rho0)
    b.set_tile(4, 0, 1, 3)
    b.set_graph_steps(k)
    b.step(4)
    b.step(2 * k)
    b.step(2 * k + 5)
    assert b.status()[1] == 4 + 4 * k + 5
    assert np.array_equal(b.get_populations()[0], fa)
    a.close(); b.close()


@pytest.mark.parametrize("scheme,eos,t", [(0, CS, 0.85), (1, CS, 0.85), (3, CS, 0.85), (4, CS, 0.95),
                                          (2, PR, 0.8)])
def test_three_step_schemes_bitwise(L, scheme, eos, t):
    gp, _ = pair(L, 300, 70, t=t, tau=0.7, scheme=scheme, sigma=0.105, eos=eos)
    rho0 = slab_rho(300, 70, eos, t, seed=8)
    ref = _run(L, gp, rho0, (2, 8, 1), 41)[0]
    for tile in [(4, 0, 1, 3), (4, 16, 1, 3)]:
        f, st, _, _ = _run(L, gp, rho0, tile, 41)
        assert st == L.LBM_OK
        assert np.array_equal(f, ref), tile


@pytest.mark.parametrize("shape", [(5, 5), (6, 9), (130, 7), (260, 5), (247, 11)])
def test_three_step_edge_shapes_vs_oracle(L, shape):
    # lattices narrower and shorter than the halo of five, one strip, ragged strips
    nx, ny = shape
    gp, op = pair(L, nx, ny, t=0.9, tau=0.9, scheme=2, sigma=0.05)
    rng = np.random.default_rng(nx * 1000 + ny)
    rho0 = np.ascontiguousarray(0.1 + 0.02 * rng.random((ny, nx)))
    f = olbm.init_equilibrium(rho0)
    lat = L.Lattice(gp, rho0)
    lat.set_populations(f, 0)
    lat.set_tile(4, 0, 1, 3)
    for n in (3, 25):
        assert olbm.step(op, f, n)[0] == 0
        lat.step(n)
        assert lat.status()[0] == L.LBM_OK
        assert rel_err(lat.moments()[0], olbm.moments(op, f)[0]) < TOL64
    lat.close()


@pytest.mark.parametrize("nx", [245, 246, 247, 253, 254, 490, 491, 493, 500])
def test_three_step_strip_edges_bitwise(L, nx):
    # widths around the strip-count thresholds (246 columns per 4-wave strip, FP64
    # edges on 64-byte boundaries)
    gp, _ = pair(L, nx, 9, t=0.8, tau=0.8, scheme=2, sigma=0.1)
    rho0 = slab_rho(nx, 9, CS, 0.8, seed=nx)
    ref = _run(L, gp, rho0, (2, 8, 1), 11)[0]
    for tile in [(4, 0, 1, 3), (4, 3, 1, 3), (8, 0, 1, 3)]:
        f, st, _, _ = _run(L, gp, rho0, tile, 11)
        assert st == L.LBM_OK
        assert np.array_equal(f, ref), tile


def test_three_step_divergence_step(L):
    # the step reported is the first with a bad node, whichever third of a launch it is
    gp, op = pair(L, 96, 80, t=0.6, tau=1.0, scheme=2, sigma=0.105, eos=PR)
    from oracle import thermo as th
    import synth
    c = th.maxwell_pr(0.6)
    rho0 = synth.droplet(96, 80, c.rho_l, c.rho_g, 20, 4.0, 0.005)
    f = olbm.init_equilibrium(rho0)
    st_o, d_o = olbm.step(op, f, 200)
    one = L.Lattice(gp, rho0)
    one.step(200)
    three = L.Lattice(gp, rho0)
    three.set_tile(4, 16, 1, 3)
    three.step(200)
    assert st_o == olbm.EDIVERGED
    assert one.status()[2] == three.status()[2]
    assert abs(three.status()[2] - d_o) <= 2
    one.close(); three.close()


def test_three_step_rejected_where_unsupported(L):
    # FP32 and FP16 arithmetic: no three-step kernel; lattices under 5 x 5; other
    # waves or depth
    for prec in (1, 2):
        gp, _ = pair(L, 64, 32, t=0.8, tau=0.8, scheme=2, sigma=0.1, precision=prec)
        lat = L.Lattice(gp, slab_rho(64, 32, CS, 0.8, seed=1))
        with pytest.raises(L.LbmError):
            lat.set_tile(4, 0, 1, 3)
        lat.close()
    gp, _ = pair(L, 4, 8, t=0.8, tau=0.8, scheme=2, sigma=0.1)
    lat = L.Lattice(gp, np.full((8, 4), 0.1))
    with pytest.raises(L.LbmError):
        lat.set_tile(4, 0, 1, 3)
    lat.close()
    gp, _ = pair(L, 64, 32, t=0.8, tau=0.8, scheme=2, sigma=0.1)
    lat = L.Lattice(gp, slab_rho(64, 32, CS, 0.8, seed=1))
    for tile in [(16, 0, 1, 3), (4, 0, 2, 3), (2, 0, 1, 3)]:
        with pytest.raises(L.LbmError):
            lat.set_tile(*tile)
    # the FP64 three-step kernel carries the MRT collision: switching to MRT keeps a
    # three-step tile, and three-step tiles are accepted under MRT
    lat.set_tile(4, 0, 1, 3)
    lat.set_mrt((1.3, 1.1, 1.2))
    assert lat.get_tile() == (4, 0, 1, 3)
    lat.set_tile(8, 0, 1, 3)
    assert lat.get_tile() == (8, 0, 1, 3)
    lat.close()
