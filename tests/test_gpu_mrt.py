"""The multiple-relaxation-time collision (lbm_set_mrt) through the C ABI against
the oracle's MRT collision (oracle/lbm_oracle.c, or_mrt_collide)."""
import numpy as np
import pytest

from oracle import lbm as olbm
from tests.gpu_common import CS, PR, pair, rel_err, slab_rho, droplet_rho

pytestmark = pytest.mark.gpu

TOL64 = 1e-10
RATES = (1.3, 1.1, 1.2)


@pytest.fixture(scope="module")
def L():
    import torch
    from paper_1204_4098_amd import lbm
    assert torch.cuda.is_available()
    lbm.lib()
    return lbm


def _mrt_pair(L, nx, ny, rates=RATES, **kw):
    gp, op = pair(L, nx, ny, **kw)
    op.mrt, op.s_e, op.s_eps, op.s_q = 1, *rates
    return gp, op


def _run(L, gp, op, rho0, checkpoints, rates=RATES, tile=None):
    lat = L.Lattice(gp, rho0)
    lat.set_mrt(rates)
    if tile:
        lat.set_tile(*tile)
    f = olbm.init_equilibrium(rho0)
    lat.set_populations(f, 0)
    errs, done = [], 0
    for n in checkpoints:
        lat.step(n - done)
        assert olbm.step(op, f, n - done)[0] == olbm.OK
        done = n
        st, _, _ = lat.status()
        assert st == L.LBM_OK
        errs.append(rel_err(lat.moments()[0], olbm.moments(op, f)[0]))
    lat.close()
    return errs


@pytest.mark.parametrize("rates", [RATES, (1.6, 0.8, 1.9)])
def test_mrt_slab_matches_oracle(L, rates):
    gp, op = _mrt_pair(L, 96, 40, rates, t=0.8, tau=0.8, scheme=2, sigma=0.1)
    errs = _run(L, gp, op, slab_rho(96, 40, CS, 0.8, seed=31), [1, 100, 1000], rates)
    print("MRT slab", rates, errs)
    assert max(errs) < TOL64, errs


@pytest.mark.parametrize("tile", [(2, 16, 1), (4, 16, 1, 2), (4, 16, 1, 3)])
def test_mrt_peng_robinson_droplet_ragged_tile(L, tile):
    gp, op = _mrt_pair(L, 130, 70, t=0.85, tau=0.9, scheme=2, sigma=0.105, eos=PR)
    errs = _run(L, gp, op, droplet_rho(130, 70, PR, 0.85, 20), [1, 50, 500], tile=tile)
    assert max(errs) < TOL64, errs


def test_mrt_f32_two_step_bitwise(L):
    """FP32 deviation storage: the two-step kernel rounds its intermediate step to
    storage as the one-step kernel does, so the two agree bit for bit."""
    gp, _ = pair(L, 200, 90, t=0.8, tau=0.7, scheme=2, sigma=0.1, precision=1)
    rho0 = slab_rho(200, 90, CS, 0.8, seed=5)
    outs = []
    for tile, graph in [((4, 0, 2), 0), ((4, 0, 2, 2), 0), ((8, 16, 1, 2), 10)]:
        lat = L.Lattice(gp, rho0)
        lat.set_mrt(RATES)
        lat.set_tile(*tile)
        if graph:
            lat.set_graph_steps(graph)
        lat.step(3)
        lat.step(34)
        outs.append(lat.save_state())
        lat.close()
    assert all(o == outs[0] for o in outs[1:])


def test_mrt_every_rate_one_over_tau_is_bgk(L):
    tau = 0.7
    gp, _ = pair(L, 128, 32, t=0.85, tau=tau, scheme=2, sigma=0.1)
    rho0 = slab_rho(128, 32, CS, 0.85, seed=4)
    a = L.Lattice(gp, rho0)
    a.step(300)
    b = L.Lattice(gp, rho0)
    b.set_mrt((1 / tau, 1 / tau, 1 / tau))
    b.step(300)
    assert rel_err(b.moments()[0], a.moments()[0]) < 1e-12
    a.close(); b.close()


def test_mrt_tiles_and_graphs_bitwise(L):
    gp, _ = pair(L, 200, 90, t=0.8, tau=0.7, scheme=2, sigma=0.1)
    rho0 = slab_rho(200, 90, CS, 0.8, seed=3)
    outs = []
    for tile, graph in [((1, 4, 1), 0), ((4, 0, 2), 0), ((16, 7, 1), 0), ((2, 0, 2), 10),
                        ((4, 0, 2, 2), 0), ((8, 5, 1, 2), 0), ((4, 32, 1, 2), 10), ((8, 0, 2, 2), 12),
                        ((4, 0, 1, 3), 0), ((8, 16, 1, 3), 0), ((4, 0, 1, 3), 10), ((4, 5, 1, 3), 12)]:
        lat = L.Lattice(gp, rho0)
        lat.set_mrt(RATES)
        lat.set_tile(*tile)
        if graph:
            lat.set_graph_steps(graph)
        lat.step(3)
        lat.step(34)
        outs.append(lat.save_state())
        lat.close()
    assert all(o == outs[0] for o in outs[1:])


def test_mrt_f32_deviations_vs_oracle(L):
    gp, op = _mrt_pair(L, 96, 40, t=0.8, tau=0.8, scheme=2, sigma=0.1, precision=1)
    lat = L.Lattice(gp, slab_rho(96, 40, CS, 0.8, seed=21))
    lat.set_mrt(RATES)
    f = olbm.init_equilibrium(slab_rho(96, 40, CS, 0.8, seed=21))
    lat.set_populations(f, 0)
    lat.step(1000)
    assert olbm.step(op, f, 1000)[0] == olbm.OK
    err = rel_err(lat.moments()[0], olbm.moments(op, f)[0])
    print("MRT FP32 deviations, node error after 1000 steps", err)
    assert err < 1e-4
    lat.close()


def test_mrt_arguments(L):
    gp, _ = pair(L, 64, 32, t=0.8, tau=0.8, scheme=0)
    rho0 = slab_rho(64, 32, CS, 0.8)
    lat = L.Lattice(gp, rho0)
    with pytest.raises(L.LbmError) as e:
        lat.set_mrt(RATES)                         # Shan-Chen: the improved scheme only
    assert e.value.status == L.LBM_ENOTSUP
    lat.close()
    gp, _ = pair(L, 64, 32, t=0.8, tau=0.8, scheme=2, sigma=0.1)
    lat = L.Lattice(gp, rho0)
    for bad in [(0.0, 1.0, 1.0), (1.0, 2.0, 1.0), (1.0, 1.0, float("nan"))]:
        with pytest.raises(L.LbmError) as e:
            lat.set_mrt(bad)
        assert e.value.status == L.LBM_EINVAL
    lat.set_tile(4, 0, 2, 2)
    lat.set_mrt(RATES)
    assert lat.get_tile() == (4, 0, 2, 2)          # the two-step kernel carries MRT
    lat.set_tile(4, 0, 1, 3)                       # and the FP64 three-step kernel
    lat.set_mrt((1.2, 1.2, 1.2))
    assert lat.get_tile() == (4, 0, 1, 3)
    lat.set_mrt(None)
    lat.close()
    gp, _ = pair(L, 64, 32, t=0.8, tau=0.8, scheme=2, sigma=0.1, precision=1)
    lat = L.Lattice(gp, rho0)
    lat.set_mrt(RATES)
    with pytest.raises(L.LbmError) as e:
        lat.set_tile(4, 0, 1, 3)                   # FP32 arithmetic: no three-step kernel
    assert e.value.status == L.LBM_ENOTSUP
    lat.close()


BATCH_RUNS = [(96, 32, 0.8, 0.8, 0.10, (1.3, 1.1, 1.2)), (200, 48, 0.7, 1.1, 0.05, (1.6, 0.8, 1.9)),
              (64, 16, 0.9, 0.6, 0.15, (1.0, 1.5, 1.1)), (130, 40, 0.75, 1.4, 0.0, (1.2, 1.2, 1.2)),
              (513, 17, 0.8, 0.9, 0.2, (1.7, 0.6, 1.4))]


def _batch_runs(L, prec):
    gps, rhos, rates = [], [], []
    for i, (nx, ny, t, tau, sigma, r) in enumerate(BATCH_RUNS):
        gp, _ = pair(L, nx, ny, t=t, tau=tau, scheme=2, sigma=sigma, precision=prec)
        gps.append(gp)
        rhos.append(slab_rho(nx, ny, CS, t, seed=40 + i))
        rates.append(r)
    return gps, rhos, rates


@pytest.mark.parametrize("prec", [0, 1])
def test_mrt_batch_equals_single_lattices_bitwise(L, prec):
    # per-run rates through lbm_batch_set_mrt: every run of every batch tile (one
    # and two steps per launch, graphs with a remainder) equals a single lattice
    # with the same rates
    gps, rhos, rates = _batch_runs(L, prec)
    ref = []
    for gp, rho, r in zip(gps, rhos, rates):
        lat = L.Lattice(gp, rho)
        lat.set_mrt(r)
        lat.step(37)
        ref.append(lat.get_populations()[0].tobytes())
        lat.close()
    for tile, graph in [((1, 4, 1, 1), 0), ((2, 0, 2, 1), 0), ((2, 0, 2, 2), 0), ((4, 32, 1, 2), 0),
                        ((2, 0, 1, 2), 10)]:
        b = L.Batch(gps, rhos)
        b.set_mrt(rates)
        b.set_tile(*tile)
        if graph:
            b.set_graph_steps(graph)
        b.step(3)
        b.step(34)
        got = [b.get_populations(i).tobytes() for i in range(len(gps))]
        b.close()
        assert got == ref, (prec, tile)


def test_mrt_batch_arguments_and_reset(L):
    gps, rhos, rates = _batch_runs(L, 0)
    bgk = L.Batch(gps, rhos)
    bgk.step(20)
    want = [bgk.get_populations(i).tobytes() for i in range(len(gps))]
    bgk.close()
    b = L.Batch(gps, rhos)
    for bad in [(0.0, 1.0, 1.0), (1.0, 2.0, 1.0), (1.0, 1.0, float("nan"))]:
        with pytest.raises(L.LbmError) as e:
            b.set_mrt(bad)
        assert e.value.status == L.LBM_EINVAL
    b.set_mrt(rates)
    b.set_tile(2, 0, 2, 2)
    b.set_mrt(None)                                  # back to BGK before any step
    b.step(20)
    assert [b.get_populations(i).tobytes() for i in range(len(gps))] == want
    b.close()
    gp_sc, _ = pair(L, 64, 32, t=0.8, tau=0.8, scheme=0)
    b = L.Batch(gps[:2] + [gp_sc], rhos[:2] + [slab_rho(64, 32, CS, 0.8)])
    with pytest.raises(L.LbmError) as e:
        b.set_mrt(RATES)                             # one Shan-Chen run: improved scheme only
    assert e.value.status == L.LBM_ENOTSUP
    b.close()
    gps16, rhos16, _ = _batch_runs(L, 2)
    b = L.Batch(gps16, rhos16)
    with pytest.raises(L.LbmError) as e:
        b.set_mrt(RATES)                             # FP16 storage
    assert e.value.status == L.LBM_ENOTSUP
    b.close()
