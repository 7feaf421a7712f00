"""ctypes wrapper over the C oracle (TEST INFRASTRUCTURE ONLY).

Layout of populations: float64 array of shape (9, ny, nx), direction first,
x fastest.  Directions e0=(0,0), e1=(1,0), e2=(0,1), e3=(-1,0), e4=(0,-1),
e5=(1,1), e6=(-1,1), e7=(-1,-1), e8=(1,-1).
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

from . import build as _build

EOS_CS, EOS_PR = 0, 1
SCHEME_SC, SCHEME_EDM, SCHEME_IMPROVED, SCHEME_EDM_MODIFIED, SCHEME_LADD = 0, 1, 2, 3, 4
OK, EINVAL, EPSI, EDIVERGED = 0, -1, -2, -3

EX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
EY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])
W = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)


class _Params(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("tau", C.c_double), ("G", C.c_double),
                ("eos", C.c_int32), ("a", C.c_double), ("b", C.c_double), ("R", C.c_double),
                ("T", C.c_double), ("omega", C.c_double), ("Tc", C.c_double),
                ("scheme", C.c_int32), ("sigma", C.c_double), ("mrt", C.c_int32),
                ("s_e", C.c_double), ("s_eps", C.c_double), ("s_q", C.c_double)]


@dataclass
class Params:
    nx: int
    ny: int
    tau: float = 1.0
    G: float = -1.0
    eos: int = EOS_CS
    a: float = 1.0
    b: float = 4.0
    R: float = 1.0
    T: float = 0.0
    omega: float = 0.0
    Tc: float = 0.0
    scheme: int = SCHEME_IMPROVED
    sigma: float = 0.0
    mrt: int = 0            # 1: multiple-relaxation-time collision (improved scheme only)
    s_e: float = 1.0
    s_eps: float = 1.0
    s_q: float = 1.0

    def c(self) -> _Params:
        return _Params(self.nx, self.ny, self.tau, self.G, self.eos, self.a, self.b, self.R,
                       self.T, self.omega, self.Tc, self.scheme, self.sigma, self.mrt, self.s_e,
                       self.s_eps, self.s_q)


_lib = None
_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
            _build.build()
        L = C.CDLL(path)
        P = C.POINTER(_Params)
        L.or_p_eos.argtypes = [P, C.c_double]; L.or_p_eos.restype = C.c_double
        L.or_psi.argtypes = [P, C.c_double, C.POINTER(C.c_double)]; L.or_psi.restype = C.c_int
        L.or_feq.argtypes = [C.c_double, C.c_double, C.c_double, _dp]; L.or_feq.restype = None
        L.or_interaction_force.argtypes = [P, _dp, _dp, _dp]; L.or_interaction_force.restype = None
        L.or_forcing.argtypes = [P, C.c_double, C.c_double, C.c_double, C.c_double, C.c_double,
                                 C.c_double, C.POINTER(C.c_double), C.POINTER(C.c_double), _dp]
        L.or_forcing.restype = None
        L.or_init_equilibrium.argtypes = [C.c_int32, C.c_int32, _dp, C.c_void_p, C.c_void_p, _dp]
        L.or_init_equilibrium.restype = None
        L.or_step.argtypes = [P, _dp, C.c_int64, C.POINTER(C.c_int64)]; L.or_step.restype = C.c_int
        L.or_moments.argtypes = [P, _dp, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        L.or_moments.restype = C.c_int
        L.or_mass.argtypes = [C.c_int32, C.c_int32, _dp, C.POINTER(C.c_double),
                              C.POINTER(C.c_int64)]
        L.or_mass.restype = None
        L.or_mrt_row.argtypes = [C.c_int, C.c_int]; L.or_mrt_row.restype = C.c_double
        L.or_mrt_collide.argtypes = [P, _dp, C.c_double, C.c_double, C.c_double, C.c_double,
                                     C.c_double, C.c_double, _dp]
        L.or_mrt_collide.restype = None
        _lib = L
    return _lib


def p_eos(p: Params, rho: float) -> float:
    return lib().or_p_eos(C.byref(p.c()), rho)


def psi(p: Params, rho: float):
    out = C.c_double()
    st = lib().or_psi(C.byref(p.c()), rho, C.byref(out))
    return out.value if st == OK else None


def mrt_matrix() -> np.ndarray:
    """The 9 x 9 moment matrix of the MRT collision (rows = moments)."""
    return np.array([[lib().or_mrt_row(k, a) for a in range(9)] for k in range(9)])


def mrt_collide(p: Params, f9, rho, ux, uy, Fx, Fy, psi2) -> np.ndarray:
    """Post-collision populations of one node under the MRT collision."""
    out = np.zeros(9)
    lib().or_mrt_collide(C.byref(p.c()), np.ascontiguousarray(f9, dtype=np.float64), rho, ux, uy,
                         Fx, Fy, psi2, out)
    return out


def feq(rho: float, ux: float, uy: float) -> np.ndarray:
    out = np.zeros(9)
    lib().or_feq(rho, ux, uy, out)
    return out


def forcing(p: Params, rho, ux, uy, Fx, Fy, psi2):
    """(u_eq, F_a) of the configured scheme at one node."""
    Fa = np.zeros(9)
    ex, ey = C.c_double(), C.c_double()
    lib().or_forcing(C.byref(p.c()), rho, ux, uy, Fx, Fy, psi2, C.byref(ex), C.byref(ey), Fa)
    return (ex.value, ey.value), Fa


def interaction_force(p: Params, psi_field: np.ndarray):
    psi_field = np.ascontiguousarray(psi_field, dtype=np.float64)
    Fx = np.zeros_like(psi_field); Fy = np.zeros_like(psi_field)
    lib().or_interaction_force(C.byref(p.c()), psi_field, Fx, Fy)
    return Fx, Fy


def init_equilibrium(rho0: np.ndarray, ux0=None, uy0=None) -> np.ndarray:
    rho0 = np.ascontiguousarray(rho0, dtype=np.float64)
    ny, nx = rho0.shape
    f = np.zeros((9, ny, nx))
    ux = None if ux0 is None else np.ascontiguousarray(ux0, dtype=np.float64)
    uy = None if uy0 is None else np.ascontiguousarray(uy0, dtype=np.float64)
    lib().or_init_equilibrium(nx, ny, rho0, None if ux is None else ux.ctypes.data,
                              None if uy is None else uy.ctypes.data, f)
    return f


def step(p: Params, f: np.ndarray, nsteps: int):
    """Advance f in place; returns (status, diverged_at)."""
    assert f.shape == (9, p.ny, p.nx) and f.dtype == np.float64 and f.flags.c_contiguous
    d = C.c_int64(-1)
    st = lib().or_step(C.byref(p.c()), f, int(nsteps), C.byref(d))
    return st, d.value


def moments(p: Params, f: np.ndarray):
    """(rho, vx, vy, p) fields, each (ny, nx); raises on an invalid state."""
    out = [np.zeros((p.ny, p.nx)) for _ in range(4)]
    st = lib().or_moments(C.byref(p.c()), np.ascontiguousarray(f), *[o.ctypes.data for o in out])
    if st != OK:
        raise RuntimeError(f"oracle moments failed: {st}")
    return tuple(out)


def mass(f: np.ndarray):
    """(double sum, fixed-point sum as Python int) of rho over all nodes."""
    _, ny, nx = f.shape
    m = C.c_double()
    lohi = (C.c_int64 * 2)()
    lib().or_mass(nx, ny, np.ascontiguousarray(f), C.byref(m), lohi)
    fixed = (lohi[1] << 64) + (lohi[0] & ((1 << 64) - 1))
    return m.value, fixed
