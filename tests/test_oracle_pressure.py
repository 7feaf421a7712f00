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
