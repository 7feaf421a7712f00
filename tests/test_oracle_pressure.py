"""Pins of the flat-interface normal pressure (Eqs. 25 and 35) in the oracle."""
from functools import lru_cache

import numpy as np
import pytest

import synth
from oracle import lbm
from oracle import pressure as pr
from oracle import thermo as th


def _params(t, sigma, tau=1.0, nx=128):
    Tc, _ = th.critical_cs()
    return lbm.Params(nx=nx, ny=3, tau=tau, scheme=lbm.SCHEME_IMPROVED, sigma=sigma, T=t * Tc)


@lru_cache(maxsize=None)
def _equilibrium(t, sigma, tau, steps=100000, nx=64):
    """Noise-free flat interface run by the oracle to equilibrium; the y-mean profile."""
    p = _params(t, sigma, tau, nx)
    c = th.maxwell_cs(t)
    f = lbm.init_equilibrium(synth.slab(nx, 3, c.rho_l, c.rho_g, nx / 4, 3 * nx / 4, 2.0, 0.0))
    st, _ = lbm.step(p, f, steps)
    assert st == lbm.OK
    return p, lbm.moments(p, f)[0].mean(axis=0)


def test_uniform_density_gives_the_eos_pressure():
    # no gradients: P_n = rho c_s^2 + G psi^2 / 2 = p_EOS (Eqs. 5 and 8)
    p = _params(0.8, 0.1, nx=8)
    for rho in (0.01, 0.1, 0.3):
        got = pr.normal_pressure(p, np.full(8, rho))
        assert np.all(np.abs(got - lbm.p_eos(p, rho)) < 1e-15 * max(1.0, rho))


@pytest.mark.parametrize("sigma,tau", [(0.0, 1.0), (0.05, 0.7), (0.1, 1.0), (0.105, 1.3)])
def test_equilibrium_interface_has_constant_normal_pressure(sigma, tau):
    # at equilibrium the normal pressure is the same on both sides and across the
    # interface: with the Eq. (35) term it is constant to rounding; dropping the term
    # or flipping its sign leaves a variation of the order of the term itself
    p, rho = _equilibrium(0.8, sigma, tau)
    P = pr.normal_pressure(p, rho)
    psi = pr.psi_profile(p, rho)
    # size of the interface term (G c^4 / 12) beta psi psi'' of Eq. (25)
    scale = np.abs(p.G / 12 * pr.BETA * psi * (np.roll(psi, -1) - 2 * psi + np.roll(psi, 1))).max()
    assert np.ptp(P) < 1e-9 * scale, (np.ptp(P), scale)
    if sigma > 0:
        for wrong in (0.0, -sigma, 2 * sigma):
            q = lbm.Params(**{**p.__dict__, "sigma": wrong})
            assert np.ptp(pr.normal_pressure(q, rho)) > 0.05 * scale


@pytest.mark.parametrize("sigma", [0.0, 0.0625, 0.1])
def test_bulk_pressure_is_the_mechanical_stability_solution(sigma):
    # the constant P_n is p0 of Eq. (26) with eps = -2(alpha + 24 G sigma)/beta = 16 sigma
    # (second-order theory; the lattice profile carries higher-order error)
    p, rho = _equilibrium(0.8, sigma, 1.0)
    P = pr.normal_pressure(p, rho)
    m = th.mechanical(th.cs_default(), p.T, 16 * sigma)
    assert abs(P.mean() / m.p0 - 1) < 0.01, (P.mean(), m.p0)
    assert abs(rho.min() / m.rho_g - 1) < 0.02 and abs(rho.max() / m.rho_l - 1) < 0.002


def test_other_schemes_are_rejected():
    p = _params(0.8, 0.0)
    p.scheme = lbm.SCHEME_EDM
    with pytest.raises(ValueError):
        pr.normal_pressure(p, np.full(8, 0.1))


def test_surface_tension_of_a_uniform_state_is_zero_and_linear_in_sigma():
    p = _params(0.8, 0.1, nx=8)
    assert pr.surface_tension(p, np.full(8, 0.2)) == 0.0
    _, rho = _equilibrium(0.8, 0.05, 1.0)
    g = [pr.surface_tension(_params(0.8, s, nx=64), rho) for s in (0.0, 0.05, 0.1)]
    # same profile: gamma is kappa(sigma) times one integral, kappa = 1/6 + 2 sigma at G = -1
    assert abs((g[2] - g[0]) / (g[1] - g[0]) - 2.0) < 1e-12
    assert abs(g[1] / g[0] - (1 / 6 + 0.1) / (1 / 6)) < 1e-12


def _laplace_slope(t, sigma, radii=(10, 14, 20), n=56, steps=5000):
    """Slope of the pressure jump p_in - p_out (p = p_EOS of the centre and corner
    3x3 means) against 1/R (equimolar radius) over noise-free oracle droplets."""
    Tc, _ = th.critical_cs()
    c = th.maxwell_cs(t)
    inv, dp = [], []
    for r in radii:
        p = lbm.Params(nx=n, ny=n, tau=1.0, scheme=lbm.SCHEME_IMPROVED, sigma=sigma, T=t * Tc)
        f = lbm.init_equilibrium(synth.droplet(n, n, c.rho_l, c.rho_g, r, 2.0, 0.0, synth.BASE_SEED))
        assert lbm.step(p, f, steps)[0] == lbm.OK
        rho, _, _, pp = lbm.moments(p, f)
        h = n // 2
        rin, rout = rho[h, h], rho[0, 0]
        inv.append(1.0 / np.sqrt((rho - rout).sum() / (np.pi * (rin - rout))))
        dp.append(pp[h - 1:h + 2, h - 1:h + 2].mean() - pp[:3, :3].mean())
    return np.polyfit(inv, dp, 1)[0]


@pytest.mark.parametrize("sigma", [0.0, 0.1])
def test_flat_surface_tension_matches_the_laplace_law(sigma):
    # the mechanical gamma of a flat interface (kappa = -G/6 plus Eq. (35)'s 2 G^2 sigma)
    # against the slope of Laplace's law over droplets, same temperature and sigma.
    # Measured (0.85 Tc, radii 10-20): Laplace / flat = 0.948 (sigma 0) and 0.991 (0.1);
    # sigma = 0.1 raises gamma 1.92x (flat) and 2.00x (Laplace).  A kappa of -G/4 or
    # -G/12, or the sigma term dropped or doubled, moves the ratio by 30 % or more at
    # one of the two sigmas.
    t = 0.85
    _, rho = _equilibrium(t, sigma, 1.0, steps=20000)
    g_flat = pr.surface_tension(_params(t, sigma, nx=64), rho)
    g_lap = _laplace_slope(t, sigma)
    print(f"sigma {sigma}: flat {g_flat:.4e}, Laplace {g_lap:.4e}, ratio {g_lap / g_flat:.4f}")
    assert abs(g_lap / g_flat - 1) < 0.08
