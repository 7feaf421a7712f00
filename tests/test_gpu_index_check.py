"""The index-checked build (liblbm_hip_check.so, LBM_CHECK_INDEX): every global
load and store of the step, copy and mass kernels is checked against its
lattice's buffer and every tile shape against the kernel's limits.  The tests
drive edge shapes, every tile family, the batch (item lists and the balanced
schedule), frozen runs, MRT (every tile family) and the diagnostics, and require zero violations."""
import ctypes as C

import numpy as np
import pytest

import synth
from oracle import thermo as th
from tests.gpu_common import CS, PR, pair, slab_rho

pytestmark = pytest.mark.gpu


@pytest.fixture
def CL(monkeypatch):
    import torch
    from paper_1204_4098_amd import lbm
    assert torch.cuda.is_available()
    chk = lbm.load(lbm.LIB_CHECK_PATH)
    monkeypatch.setattr(lbm, "_lib", chk)
    _faults(lbm)                      # start from zero
    return lbm


def _faults(L):
    n = C.c_uint64()
    assert L.lib().lbm_debug_index_faults(C.byref(n)) == L.LBM_OK
    return n.value


ONE = [(1, 1, 2), (1, 4, 1), (2, 0, 2), (4, 7, 2), (16, 0, 1), (8, 128, 2)]
TWO = [(4, 0, 2, 2), (4, 1, 1, 2), (8, 5, 2, 2), (8, 0, 1, 2)]
THREE = [(4, 0, 1, 3), (4, 1, 1, 3), (4, 64, 1, 3), (8, 0, 1, 3)]   # FP64 collision arithmetic, >= 5 x 5


@pytest.mark.parametrize("prec", [0, 1, 2, 3])
def test_single_lattice_tiles_in_bounds(CL, prec):
    L = CL
    for nx, ny in [(3, 3), (5, 4), (5, 5), (130, 7), (260, 5), (300, 70), (257, 129)]:
        gp, _ = pair(L, nx, ny, t=0.9, tau=0.9, scheme=2, sigma=0.05, precision=prec)
        rho0 = np.ascontiguousarray(0.1 + 0.02 * np.random.default_rng(nx + ny).random((ny, nx)))
        three = THREE if prec in (0, 3) and nx >= 5 and ny >= 5 else []
        for tile in ONE + TWO + three:
            lat = L.Lattice(gp, rho0)
            lat.set_tile(*tile)
            lat.step(5)
            lat.moments()
            lat.mass()
            lat.close()
    assert _faults(L) == 0


def test_batch_frozen_mrt_and_diagnostics_in_bounds(CL):
    L = CL
    specs = [(64, 16, 0.8, CS), (96, 32, 0.7, CS), (3, 3, 0.9, CS), (513, 17, 0.8, CS), (130, 20, 0.8, PR)]
    gps, rhos = [], []
    for i, (nx, ny, t, eos) in enumerate(specs):
        gp, _ = pair(L, nx, ny, t=t, tau=1.0, scheme=2, sigma=0.1, eos=eos)
        gps.append(gp)
        rhos.append(slab_rho(nx, ny, eos, t, seed=synth.BASE_SEED, stream=i) if nx > 3 else
                    np.full((ny, nx), 0.1))
    gp_bad, _ = pair(L, 96, 80, t=0.6, tau=1.0, scheme=2, sigma=0.105, eos=PR)
    c = th.maxwell_pr(0.6)
    gps.append(gp_bad)
    rhos.append(synth.droplet(96, 80, c.rho_l, c.rho_g, 20, 4.0, 0.005))
    for tile in [(1, 4, 2), (4, 0, 2), (2, 8, 1), (4, 0, 2, 2), (8, 32, 1, 2), (2, 0, 2, 2)]:
        b = L.Batch(gps, rhos)
        b.set_tile(*tile)
        b.set_graph_steps(10)
        b.step(215)                       # the last run diverges early and is frozen
        b.coexistence()
        for i in range(len(gps)):
            b.moments(i, check=False)
        b.close()
    mrt_gps = [g for g in gps if g.scheme == 2]
    mrt_rhos = [r for g, r in zip(gps, rhos) if g.scheme == 2]
    for tile in [(1, 4, 2), (4, 0, 2), (4, 0, 2, 2), (2, 8, 1, 2)]:
        b = L.Batch(mrt_gps, mrt_rhos)
        b.set_mrt((1.3, 1.1, 1.2))
        b.set_tile(*tile)
        b.step(9)
        b.close()
    gp, _ = pair(L, 130, 70, t=0.85, tau=0.9, scheme=2, sigma=0.105)
    lat = L.Lattice(gp, slab_rho(130, 70, CS, 0.85))
    lat.set_mrt((1.3, 1.1, 1.2))
    for tile in ONE + TWO + THREE:
        lat.set_tile(*tile)
        lat.step(4)
    lat.flat_profile(pressure=False)    # p_n is not defined for MRT; the column means are
    lat.surface_tension()
    b0, b1, cur = lat.device_buffers()
    fixed, m = (C.c_int64 * 2)(), C.c_double()
    assert L.lib().lbm_mass_noalloc(b1 if cur else b0, 130, 70, 0, 0.0, lat.stream.cuda_stream, fixed,
                                    C.byref(m)) == L.LBM_OK
    lat.close()
    assert _faults(L) == 0


def test_release_build_has_no_checks():
    from paper_1204_4098_amd import lbm
    n = C.c_uint64()
    assert lbm.lib().lbm_debug_index_faults(C.byref(n)) == lbm.LBM_ENOTSUP
