"""Parity of the HIP fused step (through the C ABI) with the FP64 oracle."""
import numpy as np
import pytest

from oracle import lbm as olbm
from tests.gpu_common import CS, PR, droplet_rho, pair, rel_err, slab_rho

pytestmark = pytest.mark.gpu

TOL64 = 1e-10   # relative density tolerance, FP64 path


@pytest.fixture(scope="module")
def L():
    import torch
    from paper_1204_4098_amd import lbm
    assert torch.cuda.is_available()
    lbm.lib()
    return lbm


def _run_both(L, gp, op, rho0, checkpoints, tile=None):
    f = olbm.init_equilibrium(rho0)
    lat = L.Lattice(gp, rho0)
    lat.set_populations(f, 0)
    if tile:
        lat.set_tile(*tile)
    done = 0
    errs = []
    for c in checkpoints:
        assert olbm.step(op, f, c - done)[0] == 0
        lat.step(c - done)
        done = c
        st, n, div = lat.status()
        assert st == L.LBM_OK and n == c and div == -1
        rho = lat.moments()[0]
        ref = olbm.moments(op, f)[0]
        errs.append(rel_err(rho, ref))
    g, _ = lat.get_populations()
    lat.close()
    return errs, g, f


@pytest.mark.parametrize("sigma", [0.0, 0.1])
def test_config0_slab_10000_steps(L, sigma):
    # 64 x 32, C-S at 0.8 Tc, tau = 1, improved scheme, +-1 % seeded noise, 10,000 steps
    gp, op = pair(L, 64, 32, t=0.8, tau=1.0, scheme=2, sigma=sigma)
    rho0 = slab_rho(64, 32, CS, 0.8)
    errs, g, f = _run_both(L, gp, op, rho0, [1, 10, 100, 1000, 10000])
    print("config0 sigma", sigma, "errors", errs, flush=True)
    assert max(errs) < TOL64
    assert np.max(np.abs(g - f)) < 1e-10 * np.max(np.abs(f))


@pytest.mark.parametrize("scheme", [0, 1, 2, 3, 4])
@pytest.mark.parametrize("tau", [0.6, 1.0, 1.5])
def test_schemes_ragged_tiles(L, scheme, tau):
    # ragged 67 x 29 lattice cut into 1-wave strips of 8 rows: several tiles, ragged tails;
    # Ladd's scheme (4) is stable on this interface only closer to Tc
    t = 0.95 if scheme == 4 else 0.85
    gp, op = pair(L, 67, 29, t=t, tau=tau, scheme=scheme, sigma=0.105)
    rho0 = slab_rho(67, 29, CS, t, noise=0.01, seed=7)
    errs, _, _ = _run_both(L, gp, op, rho0, [1, 50, 300], tile=(1, 8))
    assert max(errs) < TOL64, errs


@pytest.mark.parametrize("scheme", [0, 1, 2])
def test_peng_robinson_droplet(L, scheme):
    gp, op = pair(L, 96, 80, t=0.8, tau=1.0, scheme=scheme, sigma=0.105, eos=PR)
    rho0 = droplet_rho(96, 80, PR, 0.8, 20)
    errs, _, _ = _run_both(L, gp, op, rho0, [1, 20, 200, 1000], tile=(1, 16))
    assert max(errs) < TOL64, errs


def test_divergence_step_matches_oracle(L):
    # Peng-Robinson at 0.6 Tc, a sharp (W = 2) droplet: both sides leave the EOS range
    gp, op = pair(L, 96, 80, t=0.6, tau=1.0, scheme=2, sigma=0.105, eos=PR)
    from oracle import thermo as th
    import synth
    c = th.maxwell_pr(0.6)
    rho0 = synth.droplet(96, 80, c.rho_l, c.rho_g, 20, 4.0, 0.005)
    f = olbm.init_equilibrium(rho0)
    st_o, d_o = olbm.step(op, f, 200)
    lat = L.Lattice(gp, rho0)
    lat.set_populations(olbm.init_equilibrium(rho0), 0)
    lat.step(200)
    st, n, d = lat.status()
    assert st_o == olbm.EDIVERGED and st == L.LBM_EDIVERGED
    assert abs(d - d_o) <= 2, (d, d_o)


@pytest.mark.parametrize("shape", [(3, 3), (5, 4), (130, 7), (64, 128)])
def test_edge_shapes(L, shape):
    nx, ny = shape
    gp, op = pair(L, nx, ny, t=0.9, tau=0.9, scheme=2, sigma=0.05)
    rng = np.random.default_rng(nx * 1000 + ny)
    rho0 = np.ascontiguousarray(0.1 + 0.02 * rng.random((ny, nx)))
    errs, _, _ = _run_both(L, gp, op, rho0, [1, 25])
    assert max(errs) < TOL64, errs


def test_tile_shapes_bitwise_identical(L):
    gp, _ = pair(L, 200, 90, t=0.8, tau=0.7, scheme=2, sigma=0.1)
    rho0 = slab_rho(200, 90, CS, 0.8, seed=3)
    outs = []
    for tile in [(1, 4, 1), (1, 16, 2), (2, 8, 1), (4, 128, 2), (4, 5, 2), (2, 33, 1), (1, 0, 2),
                 (4, 0, 1), (2, 0, 2), (8, 0, 2), (16, 7, 1), (1, 1, 2), (2, 2, 1),
                 # two steps per launch (37 steps: 18 launches and one single step)
                 (4, 0, 2, 2), (4, 5, 1, 2), (8, 16, 2, 2), (8, 128, 1, 2), (4, 33, 2, 2)]:
        lat = L.Lattice(gp, rho0)
        lat.set_tile(*tile)
        lat.step(37)
        outs.append(lat.get_populations()[0])
        lat.close()
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])


def test_wide_strips_bitwise_identical(L):
    # 1100 columns: two 512-column strips plus a 76-column tail, or one
    # 1024-column strip plus the tail; every strip width gives the same bits
    gp, op = pair(L, 1100, 40, t=0.8, tau=0.9, scheme=2, sigma=0.1)
    rho0 = slab_rho(1100, 40, CS, 0.8, seed=4)
    outs = []
    for tile in [(1, 8, 1), (8, 0, 2), (8, 16, 1), (16, 0, 2), (16, 5, 1), (4, 0, 2),
                 (4, 0, 2, 2), (8, 0, 1, 2), (8, 7, 2, 2)]:
        lat = L.Lattice(gp, rho0)
        lat.set_tile(*tile)
        lat.step(21)
        outs.append(lat.get_populations()[0])
        lat.close()
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])
    f = olbm.init_equilibrium(rho0)
    assert olbm.step(op, f, 21)[0] == 0
    assert rel_err(outs[0], f) < TOL64


@pytest.mark.parametrize("k", [10, 12])
def test_two_step_graph_replay_bitwise(L, k):
    # graphs of k steps = k/2 two-step launches (odd for k = 10: the buffer parity flips
    # per replay), an odd eager head and tail, against single steps
    gp, _ = pair(L, 300, 70, t=0.8, tau=0.8, scheme=2, sigma=0.105)
    rho0 = slab_rho(300, 70, CS, 0.8, seed=6)
    a = L.Lattice(gp, rho0)
    a.set_tile(2, 8, 1)
    a.step(3 + 4 * k + 5)
    fa = a.get_populations()[0]
    b = L.Lattice(gp, rho0)
    b.set_tile(4, 0, 2, 2)
    b.set_graph_steps(k)
    b.step(3)
    b.step(2 * k)
    b.step(2 * k + 5)
    assert b.status()[1] == 3 + 4 * k + 5
    assert np.array_equal(b.get_populations()[0], fa)
    a.close(); b.close()


@pytest.mark.parametrize("scheme,eos,t", [(0, CS, 0.85), (1, CS, 0.85), (3, CS, 0.85), (4, CS, 0.95),
                                          (1, PR, 0.8), (2, PR, 0.8)])
def test_two_step_schemes_bitwise(L, scheme, eos, t):
    # every forcing scheme and both equations of state through two-step launches
    gp, _ = pair(L, 300, 70, t=t, tau=0.7, scheme=scheme, sigma=0.105, eos=eos)
    rho0 = slab_rho(300, 70, eos, t, seed=8)
    outs = []
    for tile in [(2, 8, 1), (4, 0, 2, 2), (8, 16, 1, 2)]:
        lat = L.Lattice(gp, rho0)
        lat.set_tile(*tile)
        lat.step(41)
        outs.append(lat.get_populations()[0])
        assert lat.status()[0] == L.LBM_OK
        lat.close()
    assert np.array_equal(outs[1], outs[0]) and np.array_equal(outs[2], outs[0])


@pytest.mark.parametrize("depth", [1, 2])
@pytest.mark.parametrize("shape", [(3, 3), (5, 4), (130, 7), (260, 5)])
def test_two_step_edge_shapes(L, shape, depth):
    nx, ny = shape
    gp, op = pair(L, nx, ny, t=0.9, tau=0.9, scheme=2, sigma=0.05)
    rng = np.random.default_rng(nx * 1000 + ny)
    rho0 = np.ascontiguousarray(0.1 + 0.02 * rng.random((ny, nx)))
    errs, _, _ = _run_both(L, gp, op, rho0, [2, 25], tile=(4, 0, depth, 2))
    assert max(errs) < TOL64, errs


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("nx", [243, 244, 250, 251, 486, 487, 493, 500])
def test_two_step_strip_edges_bitwise(L, nx, precision):
    # widths around the strip-count thresholds of the two-step kernel: a single
    # 250-column strip (every lane of a 4-wave block busy), FP64 edges rounded to
    # 64-byte boundaries, and 8-wave strips; against single steps, bit for bit
    gp, _ = pair(L, nx, 9, t=0.8, tau=0.8, scheme=2, sigma=0.1, precision=precision)
    rho0 = slab_rho(nx, 9, CS, 0.8, seed=nx)
    outs = []
    for tile in [(2, 8, 1), (4, 0, 2, 2), (4, 3, 1, 2), (8, 0, 2, 2)]:
        lat = L.Lattice(gp, rho0)
        lat.set_tile(*tile)
        lat.step(11)
        outs.append(lat.get_populations()[0])
        assert lat.status()[0] == L.LBM_OK
        lat.close()
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])


def test_two_step_divergence_step(L):
    # the same divergence as test_divergence_step_matches_oracle, through two-step launches:
    # the step reported is the first one with a bad node, whichever half of a launch it is
    gp, op = pair(L, 96, 80, t=0.6, tau=1.0, scheme=2, sigma=0.105, eos=PR)
    from oracle import thermo as th
    import synth
    c = th.maxwell_pr(0.6)
    rho0 = synth.droplet(96, 80, c.rho_l, c.rho_g, 20, 4.0, 0.005)
    f = olbm.init_equilibrium(rho0)
    st_o, d_o = olbm.step(op, f, 200)
    one = L.Lattice(gp, rho0)
    one.step(200)
    two = L.Lattice(gp, rho0)
    two.set_tile(4, 16, 2, 2)
    two.step(200)
    assert st_o == olbm.EDIVERGED
    assert one.status()[2] == two.status()[2]
    assert abs(two.status()[2] - d_o) <= 2
    one.close(); two.close()


def test_graph_replay_bitwise(L):
    gp, _ = pair(L, 128, 64, t=0.8, tau=1.0, scheme=2, sigma=0.1)
    rho0 = slab_rho(128, 64, CS, 0.8, seed=5)
    a = L.Lattice(gp, rho0)
    a.step(101)
    fa = a.get_populations()[0]
    b = L.Lattice(gp, rho0)
    b.set_graph_steps(10)
    b.step(3)        # eager, odd parity
    b.step(40)       # graphs of 10 from the odd buffer
    b.step(58)       # graphs again, plus an eager tail
    st, n, div = b.status()
    assert n == 101 and st == L.LBM_OK
    assert np.array_equal(b.get_populations()[0], fa)
    a.close(); b.close()


def test_moments_match_oracle(L):
    gp, op = pair(L, 48, 40, t=0.75, tau=0.8, scheme=1)
    rho0 = droplet_rho(48, 40, CS, 0.75, 10)
    f = olbm.init_equilibrium(rho0)
    olbm.step(op, f, 30)
    lat = L.Lattice(gp, rho0)
    lat.set_populations(f, 30)
    r, vx, vy, p = lat.moments()
    R, VX, VY, P = olbm.moments(op, f)
    assert rel_err(r, R) < 1e-14
    assert np.max(np.abs(vx - VX)) < 1e-15 and np.max(np.abs(vy - VY)) < 1e-15
    assert np.max(np.abs(p - P)) < 1e-15


def test_mass_fixed_point_bit_exact(L):
    gp, op = pair(L, 70, 33, t=0.8, tau=1.0, scheme=2, sigma=0.1)
    rho0 = slab_rho(70, 33, CS, 0.8, seed=9)
    f = olbm.init_equilibrium(rho0)
    lat = L.Lattice(gp, rho0)
    lat.set_populations(f, 0)
    m_gpu, fx_gpu = lat.mass()
    m_or, fx_or = olbm.mass(f)
    assert fx_gpu == fx_or
    lat.step(500)
    g, _ = lat.get_populations()
    m2, fx2 = lat.mass()
    assert fx2 == olbm.mass(g)[1]          # identical fields -> identical integer mass
    # conservation: rounding drift only
    assert abs(m2 - m_or) < 500 * 70 * 33 * 4e-16


def test_checkpoint_roundtrip_bitwise(L):
    gp, _ = pair(L, 96, 48, t=0.8, tau=0.9, scheme=2, sigma=0.1)
    rho0 = slab_rho(96, 48, CS, 0.8, seed=13)
    a = L.Lattice(gp, rho0)
    a.step(60)
    blob = a.save_state()
    a.step(60)
    fa = a.get_populations()[0]
    b = L.Lattice(gp, rho0)
    b.load_state(blob)
    assert b.status()[1] == 60
    b.step(60)
    assert np.array_equal(b.get_populations()[0], fa)
    a.close(); b.close()


def test_divergence_is_reported(L):
    gp, op = pair(L, 32, 16, t=0.8)
    rho0 = slab_rho(32, 16, CS, 0.8, noise=0.0)
    lat = L.Lattice(gp, rho0)
    f = olbm.init_equilibrium(rho0)
    f[4, 5, 6] = np.nan
    lat.set_populations(f, 7)
    lat.step(3)
    st, n, div = lat.status()
    assert st == L.LBM_EDIVERGED and div == 7 and n == 10
    # the oracle agrees on where it stopped
    assert olbm.step(op, f, 3) == (olbm.EDIVERGED, 0)
    # an initial density outside the EOS range is refused at init
    bad = rho0.copy()
    bad[0, 0] = 0.99
    with pytest.raises(L.LbmError) as e:
        L.Lattice(gp, bad)
    assert e.value.status == L.LBM_EPSI


def test_graphs_are_captured_before_stepping(L):
    # set_graph_steps captures both parities at once; later steps only replay them,
    # and a tile change recaptures at set_tile, not inside lbm_step
    gp, _ = pair(L, 128, 64, t=0.8, tau=1.0, scheme=2, sigma=0.1)
    rho0 = slab_rho(128, 64, CS, 0.8, seed=5)
    lat = L.Lattice(gp, rho0)
    assert lat.graph_captures() == 0
    lat.set_graph_steps(10)
    assert lat.graph_captures() == 2
    lat.step(3)
    lat.step(47)
    assert lat.graph_captures() == 2
    lat.set_tile(4, 0, 2, 2)
    assert lat.graph_captures() == 4
    lat.step(40)
    assert lat.graph_captures() == 4 and lat.status()[:2] == (L.LBM_OK, 90)
    lat.close()


@pytest.mark.parametrize("tile", [(1, 16, 2), (4, 0, 2, 2)])
def test_diverged_run_stays_frozen(L, tile):
    # after the step that diverged, further launches copy the state unchanged: the
    # populations read back do not depend on how many more steps were asked for
    gp, _ = pair(L, 96, 80, t=0.6, tau=1.0, scheme=2, sigma=0.105, eos=PR)
    from oracle import thermo as th
    import synth
    c = th.maxwell_pr(0.6)
    rho0 = synth.droplet(96, 80, c.rho_l, c.rho_g, 20, 4.0, 0.005)
    lat = L.Lattice(gp, rho0)
    lat.set_tile(*tile)
    lat.step(200)
    st, _, d = lat.status()
    assert st == L.LBM_EDIVERGED and 0 <= d < 200
    snaps = []
    for extra in (0, 1, 1, 2, 3):
        lat.step(extra)
        snaps.append(lat.save_state()[56:])   # raw storage after the header
    assert all(s == snaps[0] for s in snaps[1:])
    lat.close()
