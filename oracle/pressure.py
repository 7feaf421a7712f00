"""Normal pressure across a flat interface (TEST INFRASTRUCTURE ONLY: only the
test suite may import this module).

For a one-dimensional profile rho(n) along the interface normal n, Eq. (25)
gives the normal pressure tensor of the pseudopotential model up to
second-order derivatives,

    P_n = rho c_s^2 + (G c^2 / 2) psi^2 + (G c^4 / 12) [alpha psi'^2 + beta psi psi''],

with alpha = 0, beta = 3 for the nearest-neighbour (D2Q9) stencil (Sec. IV.A).
The improved forcing scheme adds 2 G^2 c^4 sigma psi_i psi_j to the pressure
tensor (Eq. 35), i.e. 2 G^2 sigma psi'^2 to P_n; sigma = 0 is Guo et al.'s
scheme, which adds nothing.  psi is Eq. (8); the derivatives are second-order
central differences on the lattice (spacing 1), periodic.

At equilibrium P_n must equal the bulk pressure everywhere across the
interface, which is the mechanical-stability condition of Eqs. (26) and (35).

Surface tension.  After Eq. (35) the paper writes the original pressure tensor
as P_b delta_ij + kappa d_i psi d_j psi, and the improved scheme adds
2 G^2 c^4 sigma to kappa.  It does not give kappa.  Reading: kappa is fixed by
the second-order expansion of Eq. (3) on this stencil,
F = -G [psi grad psi + (1/6) psi grad lap psi] (c = 1), written as the
divergence of a tensor of that form: -div(A I + kappa grad psi grad psi) = F
holds for every psi only with kappa = -G/6 (and A = G psi^2/2 + (G/12)|grad psi|^2
+ (G/6) psi lap psi).  Across a flat interface P_n - P_t = kappa psi'^2, so the
mechanical surface tension is gamma = (-G/6 + 2 G^2 sigma) int psi'^2 dn.
"""
from __future__ import annotations

import numpy as np

from . import lbm

ALPHA, BETA = 0.0, 3.0   # Sec. IV.A: nearest-neighbour interactions
CS2 = 1.0 / 3.0


def psi_profile(p: lbm.Params, rho: np.ndarray) -> np.ndarray:
    """Eq. (8) at every point of the profile."""
    out = np.empty(len(rho))
    for i, r in enumerate(rho):
        v = lbm.psi(p, float(r))
        if v is None:
            raise ValueError(f"density {r} outside the range of Eq. (8)")
        out[i] = v
    return out


def normal_pressure(p: lbm.Params, rho: np.ndarray) -> np.ndarray:
    """P_n(n) of Eq. (25) plus the improved scheme's term of Eq. (35)."""
    if p.scheme != lbm.SCHEME_IMPROVED:
        raise ValueError("Eq. (35) fixes the scheme term only for the improved scheme")
    rho = np.asarray(rho, dtype=np.float64)
    psi = psi_profile(p, rho)
    d1 = (np.roll(psi, -1) - np.roll(psi, 1)) / 2.0
    d2 = np.roll(psi, -1) - 2.0 * psi + np.roll(psi, 1)
    G = p.G
    original = rho * CS2 + 0.5 * G * psi ** 2 + (G / 12.0) * (ALPHA * d1 ** 2 + BETA * psi * d2)
    return original + 2.0 * G ** 2 * p.sigma * d1 ** 2


def surface_tension(p: lbm.Params, rho: np.ndarray) -> float:
    """gamma of one interface of a periodic flat slab: (kappa + 2 G^2 sigma) times
    the sum of psi'^2 over the profile (central differences), halved because the
    periodic slab has two interfaces; kappa = -G/6 (see the module notes)."""
    if p.scheme != lbm.SCHEME_IMPROVED:
        raise ValueError("Eq. (35) fixes the scheme term only for the improved scheme")
    psi = psi_profile(p, np.asarray(rho, dtype=np.float64))
    d1 = (np.roll(psi, -1) - np.roll(psi, 1)) / 2.0
    kappa = -p.G / 6.0 + 2.0 * p.G ** 2 * p.sigma
    return float(kappa * np.sum(d1 ** 2) / 2.0)
