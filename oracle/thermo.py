"""Thermodynamic analysis oracle (TEST INFRASTRUCTURE ONLY).

High-precision (mpmath) solvers for the coexistence densities the
pseudopotential lattice Boltzmann model is compared with:

  * equations of state: Carnahan-Starling (paper Sec. III.C, Eq. 23) and
    Peng-Robinson (not in the paper; standard form with
    alpha(T) = [1 + kappa (1 - sqrt(T/Tc))]^2,
    kappa = 0.37464 + 1.54226 w - 0.26992 w^2);
  * the critical point, from dp/drho = d2p/drho2 = 0;
  * the Maxwell construction of Eq. (7), by two independent methods:
      (i)  quadrature of  int (p0 - p) / rho^2 drho = 0  (equal area),
      (ii) equality of the chemical potential, mu(rho_l) = mu(rho_g), with
           mu written in closed form for each EOS;
  * the mechanical stability condition of Eq. (26) for any epsilon,
      int (p0 - p) psi' / psi^(1 + eps) drho = 0,
    and, for epsilon = 2, the integrated form of Eq. (30);
  * the epsilon of the improved forcing scheme, eps = -2 (alpha + 24 G sigma)
    / beta with alpha = 0, beta = 3 for nearest-neighbour interactions
    (Sec. IV.A after Eq. 25, and Sec. IV.B after Eq. 35).

Every coexistence solve works the same way: for a trial pressure p0 between
the spinodal pressures, rho_g(p0) and rho_l(p0) are the outer roots of
p(rho) = p0, and a one-dimensional residual in p0 is driven to zero.  The
potential follows Eq. (8) with c = 1: psi^2 = 2 (p - rho c_s^2) / G,
c_s^2 = 1/3.
"""
from __future__ import annotations

from dataclasses import dataclass
from functools import lru_cache

import mpmath as mp

mp.mp.dps = 30
CS2 = mp.mpf(1) / 3


class CarnahanStarling:
    """Eq. (23): p = rho R T (1 + eta + eta^2 - eta^3)/(1 - eta)^3 - a rho^2, eta = b rho / 4."""

    name = "CS"

    def __init__(self, a=1, b=4, R=1):
        self.a, self.b, self.R = mp.mpf(a), mp.mpf(b), mp.mpf(R)
        self.rho_max = 4 / self.b          # eta -> 1

    def p(self, rho, T):
        eta = self.b * rho / 4
        return rho * self.R * T * (1 + eta + eta**2 - eta**3) / (1 - eta)**3 - self.a * rho**2

    def dp(self, rho, T):
        # d/drho [rho Z(eta)] = (1 + 4 eta + 4 eta^2 - 4 eta^3 + eta^4) / (1 - eta)^4
        eta = self.b * rho / 4
        return (self.R * T * (1 + 4 * eta + 4 * eta**2 - 4 * eta**3 + eta**4) / (1 - eta)**4
                - 2 * self.a * rho)

    def mu(self, rho, T):
        # chemical potential up to a T-dependent constant:
        # RT [ln rho + (8 eta - 9 eta^2 + 3 eta^3)/(1 - eta)^3] - 2 a rho
        eta = self.b * rho / 4
        return (self.R * T * (mp.log(rho) + (8 * eta - 9 * eta**2 + 3 * eta**3) / (1 - eta)**3)
                - 2 * self.a * rho)


class PengRobinson:
    """p = rho R T/(1 - b rho) - a alpha(T) rho^2/(1 + 2 b rho - b^2 rho^2)."""

    name = "PR"

    def __init__(self, a=mp.mpf(2) / 49, b=mp.mpf(2) / 21, R=1, omega=mp.mpf("0.344")):
        self.a, self.b, self.R, self.omega = mp.mpf(a), mp.mpf(b), mp.mpf(R), mp.mpf(omega)
        self.kappa = mp.mpf("0.37464") + mp.mpf("1.54226") * self.omega \
            - mp.mpf("0.26992") * self.omega**2
        self.rho_max = 1 / self.b
        self._Tc = None
        self._alpha_one = False

    def alpha(self, T):
        if self._alpha_one:
            return mp.mpf(1)
        s = 1 + self.kappa * (1 - mp.sqrt(T / self.Tc))
        return s * s

    @property
    def Tc(self):
        if self._Tc is None:
            # the critical point of the EOS with alpha = 1 (alpha(Tc) = 1)
            self._alpha_one = True
            try:
                self._Tc, _ = critical_point(self)
            finally:
                self._alpha_one = False
        return self._Tc

    def p(self, rho, T):
        b = self.b
        return (rho * self.R * T / (1 - b * rho)
                - self.a * self.alpha(T) * rho**2 / (1 + 2 * b * rho - b**2 * rho**2))

    def dp(self, rho, T):
        b = self.b
        D = 1 + 2 * b * rho - b**2 * rho**2
        return (self.R * T / (1 - b * rho)**2
                - self.a * self.alpha(T) * 2 * rho * (1 + b * rho) / D**2)

    def mu(self, rho, T):
        b, s2 = self.b, mp.sqrt(2)
        aa = self.a * self.alpha(T)
        D = 1 + 2 * b * rho - b**2 * rho**2
        return (self.R * T * (mp.log(rho / (1 - b * rho)) + 1 / (1 - b * rho))
                + aa / (2 * s2 * b) * mp.log((1 + (1 - s2) * b * rho) / (1 + (1 + s2) * b * rho))
                - aa * rho / D)


def critical_point(eos):
    """(Tc, rho_c): solve dp/drho = 0 and d2p/drho2 = 0 in (rho, T).

    The starting guess comes from a coarse scan, so no printed value is used.
    """
    scale = eos.a / (eos.b * eos.R)

    def dmin(T):
        # the minimum over rho of dp/drho, located on a coarse grid
        rs = [eos.rho_max * mp.mpf(k) / 400 for k in range(1, 400)]
        vals = [eos.dp(r, T) for r in rs]
        i = min(range(len(vals)), key=lambda k: vals[k])
        return vals[i], rs[i]

    lo, hi = scale * mp.mpf("0.01"), scale * 2
    for _ in range(40):                     # bisection on the sign of min dp
        mid = (lo + hi) / 2
        if dmin(mid)[0] < 0:
            lo = mid
        else:
            hi = mid
    T0 = (lo + hi) / 2
    r0 = dmin(T0)[1]
    f1 = lambda r, T: eos.dp(r, T)
    f2 = lambda r, T: mp.diff(lambda s: eos.dp(s, T), r)
    r, T = mp.findroot([f1, f2], (r0, T0))
    return T, r


def _bracket_root(f, lo, hi, rtol=mp.mpf("1e-26"), maxit=400):
    """Root of f in [lo, hi] (f(lo), f(hi) of opposite sign) by the Illinois
    variant of regula falsi, with a bisection step whenever it stalls."""
    flo, fhi = f(lo), f(hi)
    if flo == 0:
        return lo
    if fhi == 0:
        return hi
    if (flo > 0) == (fhi > 0):
        raise ValueError("root not bracketed")
    side = 0
    for it in range(maxit):
        if it % 3 == 2:
            x = (lo + hi) / 2
        else:
            x = (lo * fhi - hi * flo) / (fhi - flo)
        fx = f(x)
        if fx == 0 or abs(hi - lo) <= rtol * abs(x):
            return x
        if (fx > 0) == (flo > 0):
            lo, flo = x, fx
            if side == -1:
                fhi /= 2
            side = -1
        else:
            hi, fhi = x, fx
            if side == 1:
                flo /= 2
            side = 1
    return (lo + hi) / 2


def spinodals(eos, T):
    """(rho_sp1, rho_sp2): the two zeros of dp/drho at T < Tc (local max, local min of p)."""
    n = 400
    rs = [eos.rho_max * mp.mpf(k) / n for k in range(1, n)]
    vals = [eos.dp(r, T) for r in rs]
    roots = []
    for k in range(len(rs) - 1):
        if vals[k] > 0 >= vals[k + 1] or vals[k] < 0 <= vals[k + 1]:
            roots.append(_bracket_root(lambda r: eos.dp(r, T), rs[k], rs[k + 1]))
    if len(roots) < 2:
        raise ValueError("no van der Waals loop: T >= Tc")
    return roots[0], roots[1]


def _outer_roots(eos, T, p0, sp):
    """rho_g(p0) in (0, rho_sp1) and rho_l(p0) in (rho_sp2, rho_max)."""
    r1, r2 = sp
    g = lambda r: eos.p(r, T) - p0
    lo = r1 * mp.mpf("1e-30")
    rg = _bracket_root(g, lo, r1)
    hi = r2
    step = (eos.rho_max - r2) / 2
    while g(hi + step) < 0:                 # bracket the liquid root below rho_max
        hi = hi + step
        step = step / 2
    rl = _bracket_root(g, hi, hi + step)
    return rg, rl


def _solve_p0(eos, T, residual):
    sp = spinodals(eos, T)
    pmax = eos.p(sp[0], T)
    pmin = max(eos.p(sp[1], T), pmax * mp.mpf("1e-12"))
    eps = (pmax - pmin) * mp.mpf("1e-12")
    lo, hi = pmin + eps, pmax - eps
    f = lambda p0: residual(p0, *_outer_roots(eos, T, p0, sp))
    p0 = _bracket_root(f, lo, hi, rtol=mp.mpf("1e-22"))
    rg, rl = _outer_roots(eos, T, p0, sp)
    return rl, rg, p0


@dataclass(frozen=True)
class Coexistence:
    rho_l: float
    rho_g: float
    p0: float


def maxwell_area(eos, T):
    """Method (i): int_{rho_g}^{rho_l} (p0 - p(rho)) / rho^2 drho = 0 (Eq. 7)."""
    def res(p0, rg, rl):
        return mp.quad(lambda r: (p0 - eos.p(r, T)) / r**2, [rg, (rg + rl) / 2, rl])
    rl, rg, p0 = _solve_p0(eos, T, res)
    return Coexistence(float(rl), float(rg), float(p0))


def maxwell_mu(eos, T):
    """Method (ii): mu(rho_l) = mu(rho_g) with p(rho_l) = p(rho_g) = p0."""
    def res(p0, rg, rl):
        return eos.mu(rl, T) - eos.mu(rg, T)
    rl, rg, p0 = _solve_p0(eos, T, res)
    return Coexistence(float(rl), float(rg), float(p0))


def psi2(eos, rho, T, G=-1):
    """Eq. (8), c = 1: psi^2 = 2 (p_EOS - rho c_s^2) / G.

    A model EOS defined through psi itself may supply psi2() directly, which
    avoids the cancellation of p - rho c_s^2 at very low density."""
    if hasattr(eos, "psi2"):
        return eos.psi2(rho, T, G)
    return 2 * (eos.p(rho, T) - rho * CS2) / G


def dpsi2(eos, rho, T, G=-1):
    """d(psi^2)/drho = 2 (dp/drho - c_s^2) / G, from Eq. (8)."""
    if hasattr(eos, "dpsi2"):
        return eos.dpsi2(rho, T, G)
    return 2 * (eos.dp(rho, T) - CS2) / G


def mechanical(eos, T, eps, G=-1):
    """Eq. (26): int (p0 - p) psi'/psi^(1+eps) drho = 0, psi' from Eq. (8).

    psi'/psi^(1+eps) = (d psi^2/drho) / (2 psi^(2+eps)).
    """
    G = mp.mpf(G)
    eps = mp.mpf(eps)

    def integrand(p0, r):
        # psi' / psi^(1+eps) = (d psi^2 / d rho) / (2 psi^(2+eps))
        s2 = psi2(eos, r, T, G)
        return (p0 - eos.p(r, T)) * dpsi2(eos, r, T, G) / (2 * s2 ** (1 + eps / 2))

    def res(p0, rg, rl):
        return mp.quad(lambda r: integrand(p0, r), [rg, (rg + rl) / 2, rl])
    rl, rg, p0 = _solve_p0(eos, T, res)
    return Coexistence(float(rl), float(rg), float(p0))


def mechanical_eps2_eq30(eos, T, G=-1):
    """Eq. (30), the integrated form of the epsilon = 2 condition:
    (p0 - rho c_s^2)(-1/(2 psi^2)) | - (G/2) ln psi | + int c_s^2 (-1/(2 psi^2)) drho = 0."""
    G = mp.mpf(G)

    def res(p0, rg, rl):
        term = lambda r: (p0 - r * CS2) * (-1 / (2 * psi2(eos, r, T, G)))
        lnpsi = lambda r: mp.log(psi2(eos, r, T, G)) / 2
        integral = mp.quad(lambda r: CS2 * (-1 / (2 * psi2(eos, r, T, G))), [rg, (rg + rl) / 2, rl])
        return (term(rl) - term(rg)) - G / 2 * (lnpsi(rl) - lnpsi(rg)) + integral
    rl, rg, p0 = _solve_p0(eos, T, res)
    return Coexistence(float(rl), float(rg), float(p0))


def epsilon_of_sigma(sigma, G=-1, alpha=0, beta=3):
    """eps = -2 (alpha + 24 G sigma) / beta (Sec. IV.B, after Eq. 35)."""
    return -2.0 * (alpha + 24.0 * G * sigma) / beta


def sigma_of_epsilon(eps, G=-1, alpha=0, beta=3):
    return (-eps * beta / 2.0 - alpha) / (24.0 * G)


@lru_cache(maxsize=None)
def cs_default():
    return CarnahanStarling()


@lru_cache(maxsize=None)
def pr_default():
    return PengRobinson()


@lru_cache(maxsize=None)
def critical_cs():
    T, r = critical_point(cs_default())
    return float(T), float(r)


@lru_cache(maxsize=None)
def critical_pr():
    eos = pr_default()
    return float(eos.Tc), float(critical_point_pr_rho(eos))


def critical_point_pr_rho(eos):
    eos._alpha_one = True
    try:
        _, r = critical_point(eos)
    finally:
        eos._alpha_one = False
    return r


@lru_cache(maxsize=None)
def maxwell_cs(t_over_tc: float) -> Coexistence:
    Tc, _ = critical_cs()
    return maxwell_area(cs_default(), mp.mpf(t_over_tc) * mp.mpf(Tc))


@lru_cache(maxsize=None)
def maxwell_pr(t_over_tc: float) -> Coexistence:
    eos = pr_default()
    return maxwell_area(eos, mp.mpf(t_over_tc) * eos.Tc)


@lru_cache(maxsize=None)
def mechanical_cs(t_over_tc: float, eps: float) -> Coexistence:
    Tc, _ = critical_cs()
    return mechanical(cs_default(), mp.mpf(t_over_tc) * mp.mpf(Tc), eps)


def sigma_star_cs(t_over_tc: float, tol: float = 1e-7) -> float:
    """Theory sigma* (C-S): the eps whose Eq. (26) solution has the Maxwell vapour
    density, mapped back with eps = 16 sigma (Sec. IV.B); secant iteration."""
    target = maxwell_cs(t_over_tc).rho_g
    f = lambda e: mechanical_cs(t_over_tc, float(e)).rho_g / target - 1.0
    e0, e1 = 1.6, 1.75
    f0, f1 = f(e0), f(e1)
    for _ in range(30):
        e2 = e1 - f1 * (e1 - e0) / (f1 - f0)
        if abs(e2 - e1) < tol:
            e1 = e2
            break
        e0, f0, e1, f1 = e1, f1, e2, f(e2)
    return sigma_of_epsilon(e1)
