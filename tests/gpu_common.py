"""Helpers of the GPU parity tests: the same seeded inputs go to the oracle and
to the HIP path (populations handed over bit-for-bit with set_populations)."""
import numpy as np

import synth
from oracle import lbm as olbm
from oracle import thermo as th

CS = dict(eos=0, a=1.0, b=4.0, R=1.0, omega=0.0)
PR = dict(eos=1, a=2 / 49, b=2 / 21, R=1.0, omega=0.344)


def temperature(eos, t):
    Tc = th.critical_cs()[0] if eos == 0 else th.critical_pr()[0]
    return t * Tc, Tc


def coexistence(eos, t):
    return th.maxwell_cs(t) if eos == 0 else th.maxwell_pr(t)


def pair(L, nx, ny, t=0.8, tau=1.0, scheme=2, sigma=0.0, eos=CS, precision=0, rho_ref=float("nan")):
    """(gpu lbm_params, oracle Params) with identical physical parameters."""
    T, Tc = temperature(eos["eos"], t)
    gp = L.params(nx, ny, tau=tau, G=-1.0, T=T, scheme=scheme, sigma=sigma, precision=precision,
                  rho_ref=rho_ref, **eos)
    op = olbm.Params(nx=nx, ny=ny, tau=tau, G=-1.0, T=T, Tc=Tc, scheme=scheme, sigma=sigma,
                     **{k: v for k, v in eos.items()})
    return gp, op


def slab_rho(nx, ny, eos, t, noise=0.01, seed=synth.BASE_SEED, stream=0):
    c = coexistence(eos["eos"], t)
    return synth.slab(nx, ny, c.rho_l, c.rho_g, nx / 4, 3 * nx / 4, 2.0, noise, seed, stream)


def droplet_rho(nx, ny, eos, t, r0, noise=0.005, seed=synth.BASE_SEED):
    c = coexistence(eos["eos"], t)
    return synth.droplet(nx, ny, c.rho_l, c.rho_g, r0, 2.0, noise, seed)


def rel_err(a, b):
    return float(np.max(np.abs(a - b) / np.abs(b)))


MIRROR_X = [0, 3, 2, 1, 4, 6, 5, 8, 7]   # direction index after x -> -x
MIRROR_Y = [0, 1, 4, 3, 2, 8, 7, 6, 5]   # direction index after y -> -y


def mirror_tile(win):
    """A 2w x 2w periodic lattice made of the window and its three mirror images,
    so that wrapping creates no density jump."""
    mx = win[MIRROR_X][:, :, ::-1]
    my = win[MIRROR_Y][:, ::-1, :]
    mxy = win[MIRROR_X][MIRROR_Y][:, ::-1, ::-1]
    top = np.concatenate([win, mx], axis=2)
    bot = np.concatenate([my, mxy], axis=2)
    return np.ascontiguousarray(np.concatenate([top, bot], axis=1))
