"""Surface tension of a flat interface (lbm_surface_tension) against the oracle's
formula on the same profile, and against Laplace's law over droplets run by the
batched launch (the consistency of Eq. (35)'s change of kappa with the pressure
jump of curved interfaces)."""
import numpy as np
import pytest

import synth
from oracle import lbm as olbm
from oracle import pressure as pr
from oracle import thermo as th
from tests.gpu_common import CS, pair, slab_rho

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import torch
    from paper_1204_4098_amd import lbm
    assert torch.cuda.is_available()
    lbm.lib()
    return lbm


@pytest.mark.parametrize("sigma", [0.0, 0.1])
def test_surface_tension_matches_oracle_formula(L, sigma):
    gp, op = pair(L, 96, 8, t=0.8, tau=1.0, scheme=2, sigma=sigma)
    lat = L.Lattice(gp, slab_rho(96, 8, CS, 0.8, noise=0.0))
    lat.step(3000)
    rb, _ = lat.flat_profile(pressure=False)
    g = lat.surface_tension()
    ref = pr.surface_tension(op, rb)
    assert abs(g / ref - 1) < 1e-12, (g, ref)
    lat.close()
    # other schemes: not defined by the paper
    gp, _ = pair(L, 96, 8, t=0.8, tau=1.0, scheme=1)
    lat = L.Lattice(gp, slab_rho(96, 8, CS, 0.8, noise=0.0))
    with pytest.raises(L.LbmError) as e:
        lat.surface_tension()
    assert e.value.status == L.LBM_ENOTSUP
    lat.close()


def test_laplace_law_matches_flat_surface_tension(L):
    # droplets of radius 16 .. 48 on 160^2 lattices, sigma in {0, 0.05, 0.1}, C-S 0.85 Tc,
    # tau = 1, one batched launch; slope of p_in - p_out against 1/R (equimolar radius)
    # against gamma of a flat interface at the same sigma
    t, n, radii, sigmas = 0.85, 160, (16, 24, 32, 48), (0.0, 0.05, 0.1)
    Tc = th.critical_cs()[0]
    c = th.maxwell_cs(t)
    gps, rhos = [], []
    for s in sigmas:
        for r in radii:
            gps.append(L.params(n, n, tau=1.0, T=t * Tc, scheme=L.LBM_SCHEME_IMPROVED, sigma=s, **{
                k: v for k, v in CS.items()}))
            rhos.append(synth.droplet(n, n, c.rho_l, c.rho_g, r, 2.0, 0.0, synth.BASE_SEED))
    b = L.Batch(gps, rhos)
    b.set_graph_steps(100)
    b.step(20000)
    out = []
    for k, s in enumerate(sigmas):
        inv, dp = [], []
        for j, r in enumerate(radii):
            rho, _, _, p = b.moments(k * len(radii) + j)
            h = n // 2
            rin, rout = rho[h, h], rho[0, 0]
            inv.append(1.0 / np.sqrt((rho - rout).sum() / (np.pi * (rin - rout))))
            dp.append(p[h - 1:h + 2, h - 1:h + 2].mean() - p[:3, :3].mean())
        slope, icpt = np.polyfit(inv, dp, 1)
        gp, op = pair(L, 128, 4, t=t, tau=1.0, scheme=2, sigma=s)
        lat = L.Lattice(gp, slab_rho(128, 4, CS, t, noise=0.0))
        lat.step(20000)
        g = lat.surface_tension()
        lat.close()
        print(f"sigma {s}: Laplace {slope:.4e} (intercept {icpt:.1e}), flat {g:.4e}, ratio {slope / g:.4f}",
              flush=True)
        out.append((slope, g))
        assert abs(slope / g - 1) < 0.05, (s, slope, g)
    # Eq. (35): sigma raises gamma by the same factor in both measurements
    for (sl, g) in out[1:]:
        assert abs((sl / out[0][0]) / (g / out[0][1]) - 1) < 0.05
    b.close()
