"""Thin ctypes binding of liblbm_hip.so (the C ABI in include/lbm.h).

Argument marshalling only: every step of the lattice Boltzmann update runs in
the library's HIP kernels.  PyTorch provides the device workspace (a uint8
tensor) and the HIP stream.  Function names mirror the C ABI; the classes
`Lattice` and `Batch` hold a context and its workspace together.
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np
import torch  # loaded first, so the library binds to the HIP runtime torch already holds

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm_hip.so")
LIB_CHECK_PATH = os.path.join(HERE, "liblbm_hip_check.so")   # index-checked build (tests)

LBM_OK, LBM_EINVAL, LBM_EPSI, LBM_EDIVERGED, LBM_EHIP, LBM_ENOSPACE, LBM_ENOTSUP = 0, -1, -2, -3, -4, -5, -6
LBM_EOS_CS, LBM_EOS_PR = 0, 1
LBM_SCHEME_SHANCHEN, LBM_SCHEME_EDM, LBM_SCHEME_IMPROVED, LBM_SCHEME_EDM_MODIFIED, LBM_SCHEME_LADD = 0, 1, 2, 3, 4
LBM_PREC_F64, LBM_PREC_F32DEV, LBM_PREC_F16DEV, LBM_PREC_F32DEV_F64 = 0, 1, 2, 3


class lbm_params(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("tau", C.c_double), ("G", C.c_double),
                ("eos", C.c_int32), ("a", C.c_double), ("b", C.c_double), ("R", C.c_double),
                ("T", C.c_double), ("omega", C.c_double), ("scheme", C.c_int32),
                ("sigma", C.c_double), ("precision", C.c_int32), ("rho_ref", C.c_double)]


class LbmError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        super().__init__(f"{what}: {lbm_strerror(status)} ({status})" if what else lbm_strerror(status))


_lib = None
_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)
_lp = C.POINTER(C.c_int64)
_vp = C.c_void_p
_P = C.POINTER(lbm_params)

_SIGS = {
    "lbm_strerror": (C.c_char_p, [C.c_int]),
    "lbm_critical_point": (C.c_int, [C.c_int32, C.c_double, C.c_double, C.c_double, C.c_double, _dp, _dp]),
    "lbm_maxwell": (C.c_int, [C.c_int32, C.c_double, C.c_double, C.c_double, C.c_double, C.c_double,
                              _dp, _dp, _dp]),
    "lbm_pressure": (C.c_int, [_P, C.c_double, _dp]),
    "lbm_workspace_bytes": (C.c_int, [_P, C.POINTER(C.c_size_t)]),
    "lbm_init": (C.c_int, [_P, _vp, _vp, _vp, _vp, C.c_size_t, _vp, C.POINTER(_vp)]),
    "lbm_step": (C.c_int, [_vp, C.c_int64]),
    "lbm_status": (C.c_int, [_vp, _lp, _lp]),
    "lbm_moments": (C.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "lbm_moments_device": (C.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "lbm_mass": (C.c_int, [_vp, _lp, _dp]),
    "lbm_mass_noalloc": (C.c_int, [_vp, C.c_int32, C.c_int32, C.c_int32, C.c_double, _vp, _lp, _dp]),
    "lbm_flat_profile": (C.c_int, [_vp, _vp, _vp]),
    "lbm_surface_tension": (C.c_int, [_vp, _dp]),
    "lbm_get_populations": (C.c_int, [_vp, _vp, _lp]),
    "lbm_set_populations": (C.c_int, [_vp, _vp, C.c_int64]),
    "lbm_state_bytes": (C.c_int, [_vp, C.POINTER(C.c_size_t)]),
    "lbm_save_state": (C.c_int, [_vp, _vp, C.c_size_t]),
    "lbm_load_state": (C.c_int, [_vp, _vp, C.c_size_t]),
    "lbm_tune": (C.c_int, [_vp, _ip, _ip, _ip, _ip]),
    "lbm_set_tile": (C.c_int, [_vp, C.c_int32, C.c_int32, C.c_int32, C.c_int32]),
    "lbm_get_tile": (C.c_int, [_vp, _ip, _ip, _ip, _ip]),
    "lbm_set_graph_steps": (C.c_int, [_vp, C.c_int32]),
    "lbm_graph_captures": (C.c_int, [_vp, _lp]),
    "lbm_set_mrt": (C.c_int, [_vp, _vp]),
    "lbm_device_buffers": (C.c_int, [_vp, C.POINTER(_vp), C.POINTER(_vp), _ip]),
    "lbm_get_params": (C.c_int, [_vp, _P]),
    "lbm_debug_index_faults": (C.c_int, [C.POINTER(C.c_uint64)]),
    "lbm_destroy": (C.c_int, [_vp]),
    "lbm_batch_workspace_bytes": (C.c_int, [C.c_int32, _P, C.POINTER(C.c_size_t)]),
    "lbm_batch_init": (C.c_int, [C.c_int32, _P, C.POINTER(_vp), _vp, C.c_size_t, _vp, C.POINTER(_vp)]),
    "lbm_batch_step": (C.c_int, [_vp, C.c_int64]),
    "lbm_batch_coexistence": (C.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "lbm_batch_moments": (C.c_int, [_vp, C.c_int32, _vp, _vp, _vp, _vp]),
    "lbm_batch_get_populations": (C.c_int, [_vp, C.c_int32, _vp]),
    "lbm_batch_tune": (C.c_int, [_vp, _ip, _ip, _ip, _ip]),
    "lbm_batch_set_tile": (C.c_int, [_vp, C.c_int32, C.c_int32, C.c_int32, C.c_int32]),
    "lbm_batch_get_tile": (C.c_int, [_vp, _ip, _ip, _ip, _ip]),
    "lbm_batch_set_graph_steps": (C.c_int, [_vp, C.c_int32]),
    "lbm_batch_set_mrt": (C.c_int, [_vp, _vp]),
    "lbm_batch_graph_captures": (C.c_int, [_vp, _lp]),
    "lbm_batch_nodes": (C.c_int, [_vp, _lp]),
    "lbm_batch_destroy": (C.c_int, [_vp]),
}


def load(path: str):
    """Load a build of the library and declare its C signatures; raises if it has
    not been built (there is no CPU fallback)."""
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with __graft_entry__.build() "
                           "(there is no CPU fallback)")
    L = C.CDLL(path)
    for name, (res, args) in _SIGS.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    return L


def lib():
    """The loaded library (the release build)."""
    global _lib
    if _lib is None:
        _lib = load(LIB_PATH)
    return _lib


def lbm_strerror(status: int) -> str:
    return lib().lbm_strerror(int(status)).decode()


def _check(st: int, what: str):
    if st != LBM_OK:
        raise LbmError(st, what)


def params(nx, ny, tau=1.0, G=-1.0, eos=LBM_EOS_CS, a=1.0, b=4.0, R=1.0, T=None,
           t_over_tc=None, omega=0.0, scheme=LBM_SCHEME_IMPROVED, sigma=0.0,
           precision=LBM_PREC_F64, rho_ref=math.nan) -> lbm_params:
    """Build an lbm_params; give either T (absolute) or t_over_tc."""
    if T is None:
        if t_over_tc is None:
            raise ValueError("give T or t_over_tc")
        T = t_over_tc * lbm_critical_point(eos, a, b, R, omega)[0]
    return lbm_params(int(nx), int(ny), float(tau), float(G), int(eos), float(a), float(b), float(R),
                      float(T), float(omega), int(scheme), float(sigma), int(precision), float(rho_ref))


def lbm_critical_point(eos=LBM_EOS_CS, a=1.0, b=4.0, R=1.0, omega=0.0):
    Tc, rc = C.c_double(), C.c_double()
    _check(lib().lbm_critical_point(eos, a, b, R, omega, C.byref(Tc), C.byref(rc)), "lbm_critical_point")
    return Tc.value, rc.value


def lbm_maxwell(eos, a, b, R, omega, T):
    rl, rg, p0 = C.c_double(), C.c_double(), C.c_double()
    _check(lib().lbm_maxwell(eos, a, b, R, omega, T, C.byref(rl), C.byref(rg), C.byref(p0)), "lbm_maxwell")
    return rl.value, rg.value, p0.value


def lbm_pressure(p: lbm_params, rho: float) -> float:
    out = C.c_double()
    _check(lib().lbm_pressure(C.byref(p), rho, C.byref(out)), "lbm_pressure")
    return out.value


def lbm_workspace_bytes(p: lbm_params) -> int:
    n = C.c_size_t()
    _check(lib().lbm_workspace_bytes(C.byref(p), C.byref(n)), "lbm_workspace_bytes")
    return n.value


def _f64(a, shape=None):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None and a.shape != shape:
        raise ValueError(f"expected shape {shape}, got {a.shape}")
    return a


def _ptr(a):
    return None if a is None else a.ctypes.data


def _workspace(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def _new_stream(device):
    # a non-default stream (default priority) so that HIP graphs can be captured on it
    return torch.cuda.Stream(device=device)


class Lattice:
    """One periodic lattice on the GPU (an lbm_ctx and its workspace)."""

    def __init__(self, p: lbm_params, rho0, ux0=None, uy0=None, device="cuda:0", stream=None):
        self.p = p
        shape = (p.ny, p.nx)
        rho0, ux0, uy0 = _f64(rho0, shape), _f64(ux0, shape), _f64(uy0, shape)
        self.device = torch.device(device)
        self.stream = stream if stream is not None else _new_stream(self.device)
        self.workspace = _workspace(lbm_workspace_bytes(p), self.device)
        torch.cuda.synchronize(self.device)
        h = _vp()
        _check(lib().lbm_init(C.byref(p), _ptr(rho0), _ptr(ux0), _ptr(uy0), self.workspace.data_ptr(),
                              self.workspace.numel(), self.stream.cuda_stream, C.byref(h)), "lbm_init")
        self.ctx = h

    # -- time stepping
    def step(self, n: int):
        _check(lib().lbm_step(self.ctx, int(n)), "lbm_step")

    def status(self):
        s, d = C.c_int64(), C.c_int64()
        st = lib().lbm_status(self.ctx, C.byref(s), C.byref(d))
        if st not in (LBM_OK, LBM_EDIVERGED):
            _check(st, "lbm_status")
        return st, s.value, d.value

    # -- outputs
    def moments(self, check=True):
        out = [np.empty((self.p.ny, self.p.nx)) for _ in range(4)]
        st = lib().lbm_moments(self.ctx, *[o.ctypes.data for o in out])
        if check or st not in (LBM_OK, LBM_EDIVERGED):
            _check(st, "lbm_moments")
        return tuple(out)

    def flat_profile(self, pressure: bool = True):
        """(rho_bar, p_n): y-mean density per column and the normal pressure of
        Eqs. (25)/(35) across an interface with normal x (p_n: improved scheme)."""
        rb = np.empty(self.p.nx)
        pn = np.empty(self.p.nx) if pressure else None
        _check(lib().lbm_flat_profile(self.ctx, rb.ctypes.data, None if pn is None else pn.ctypes.data),
               "lbm_flat_profile")
        return rb, pn

    def surface_tension(self) -> float:
        """gamma of a flat interface with normal x (improved scheme; see lbm.h)."""
        g = C.c_double()
        _check(lib().lbm_surface_tension(self.ctx, C.byref(g)), "lbm_surface_tension")
        return g.value

    def moments_device(self):
        """(rho, vx, vy, p) as device tensors; the library writes them on the
        lattice's stream, and the caller's current stream is made to wait for it."""
        out = [torch.empty((self.p.ny, self.p.nx), dtype=torch.float64, device=self.device) for _ in range(4)]
        _check(lib().lbm_moments_device(self.ctx, *[o.data_ptr() for o in out]), "lbm_moments_device")
        torch.cuda.current_stream(self.device).wait_stream(self.stream)
        return tuple(out)

    def mass(self):
        fixed = (C.c_int64 * 2)()
        m = C.c_double()
        _check(lib().lbm_mass(self.ctx, fixed, C.byref(m)), "lbm_mass")
        return m.value, (fixed[1] << 64) + (fixed[0] & ((1 << 64) - 1))

    def get_populations(self):
        f = np.empty((9, self.p.ny, self.p.nx))
        s = C.c_int64()
        st = lib().lbm_get_populations(self.ctx, f.ctypes.data, C.byref(s))
        if st not in (LBM_OK, LBM_EDIVERGED):
            _check(st, "lbm_get_populations")
        return f, s.value

    def set_populations(self, f, step=0):
        f = _f64(f, (9, self.p.ny, self.p.nx))
        _check(lib().lbm_set_populations(self.ctx, f.ctypes.data, int(step)), "lbm_set_populations")

    def save_state(self) -> bytes:
        n = C.c_size_t()
        _check(lib().lbm_state_bytes(self.ctx, C.byref(n)), "lbm_state_bytes")
        buf = C.create_string_buffer(n.value)
        _check(lib().lbm_save_state(self.ctx, buf, n.value), "lbm_save_state")
        return buf.raw

    def load_state(self, data: bytes):
        buf = C.create_string_buffer(data, len(data))
        _check(lib().lbm_load_state(self.ctx, buf, len(data)), "lbm_load_state")

    # -- launch shape
    def tune(self):
        """Fastest tile per lattice step: (waves, rows, depth, steps per launch)."""
        w, r, d, k = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
        _check(lib().lbm_tune(self.ctx, C.byref(w), C.byref(r), C.byref(d), C.byref(k)), "lbm_tune")
        return w.value, r.value, d.value, k.value

    def set_tile(self, waves: int, rows: int, depth: int = 2, steps: int = 1):
        _check(lib().lbm_set_tile(self.ctx, int(waves), int(rows), int(depth), int(steps)), "lbm_set_tile")

    def get_tile(self):
        w, r, d, k = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
        _check(lib().lbm_get_tile(self.ctx, C.byref(w), C.byref(r), C.byref(d), C.byref(k)), "lbm_get_tile")
        return w.value, r.value, d.value, k.value

    def set_graph_steps(self, k: int):
        """Replay steps through graphs of k steps (captured now, both parities)."""
        _check(lib().lbm_set_graph_steps(self.ctx, int(k)), "lbm_set_graph_steps")

    def graph_captures(self) -> int:
        n = C.c_int64()
        _check(lib().lbm_graph_captures(self.ctx, C.byref(n)), "lbm_graph_captures")
        return n.value

    def set_mrt(self, rates=None):
        """MRT collision with (s_e, s_eps, s_q); None restores BGK."""
        if rates is None:
            _check(lib().lbm_set_mrt(self.ctx, None), "lbm_set_mrt")
            return
        r = (C.c_double * 3)(*[float(v) for v in rates])
        _check(lib().lbm_set_mrt(self.ctx, r), "lbm_set_mrt")

    def params(self) -> lbm_params:
        """The context's parameters (rho_ref resolved to the value in use)."""
        out = lbm_params()
        _check(lib().lbm_get_params(self.ctx, C.byref(out)), "lbm_get_params")
        return out

    def rho_ref(self) -> float:
        return self.params().rho_ref

    def device_buffers(self):
        b0, b1, cur = _vp(), _vp(), C.c_int32()
        _check(lib().lbm_device_buffers(self.ctx, C.byref(b0), C.byref(b1), C.byref(cur)), "lbm_device_buffers")
        return b0.value, b1.value, cur.value

    def close(self):
        if getattr(self, "ctx", None):
            lib().lbm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def lbm_batch_workspace_bytes(ps) -> int:
    arr = (lbm_params * len(ps))(*ps)
    n = C.c_size_t()
    _check(lib().lbm_batch_workspace_bytes(len(ps), arr, C.byref(n)), "lbm_batch_workspace_bytes")
    return n.value


class Batch:
    """Many independent lattices advanced by one persistent launch per step."""

    def __init__(self, ps, rho0s, device="cuda:0", stream=None):
        self.ps = list(ps)
        n = len(self.ps)
        self._arr = (lbm_params * n)(*self.ps)
        self._rho = [_f64(r, (q.ny, q.nx)) for r, q in zip(rho0s, self.ps)]
        ptrs = (_vp * n)(*[r.ctypes.data for r in self._rho])
        self.device = torch.device(device)
        self.stream = stream if stream is not None else _new_stream(self.device)
        self.workspace = _workspace(lbm_batch_workspace_bytes(self.ps), self.device)
        torch.cuda.synchronize(self.device)
        h = _vp()
        _check(lib().lbm_batch_init(n, self._arr, ptrs, self.workspace.data_ptr(), self.workspace.numel(),
                                    self.stream.cuda_stream, C.byref(h)), "lbm_batch_init")
        self.b = h

    def step(self, n: int):
        _check(lib().lbm_batch_step(self.b, int(n)), "lbm_batch_step")

    def coexistence(self):
        n = len(self.ps)
        rl, rg = np.empty(n), np.empty(n)
        st, dv = np.empty(n, dtype=np.int32), np.empty(n, dtype=np.int64)
        _check(lib().lbm_batch_coexistence(self.b, rl.ctypes.data, rg.ctypes.data, st.ctypes.data,
                                           dv.ctypes.data), "lbm_batch_coexistence")
        return rl, rg, st, dv

    def moments(self, run: int, check=True):
        """(rho, vx, vy, p) of one run; check=False also returns the frozen state
        of a diverged run instead of raising."""
        q = self.ps[run]
        out = [np.empty((q.ny, q.nx)) for _ in range(4)]
        st = lib().lbm_batch_moments(self.b, int(run), *[o.ctypes.data for o in out])
        if check or st not in (LBM_OK, LBM_EDIVERGED):
            _check(st, "lbm_batch_moments")
        return tuple(out)

    def get_populations(self, run: int, check=True):
        q = self.ps[run]
        f = np.empty((9, q.ny, q.nx))
        st = lib().lbm_batch_get_populations(self.b, int(run), f.ctypes.data)
        if check or st not in (LBM_OK, LBM_EDIVERGED):
            _check(st, "lbm_batch_get_populations")
        return f

    def tune(self):
        """Fastest tile per lattice step: (waves, rows, depth, steps per launch)."""
        w, r, d, k = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
        _check(lib().lbm_batch_tune(self.b, C.byref(w), C.byref(r), C.byref(d), C.byref(k)), "lbm_batch_tune")
        return w.value, r.value, d.value, k.value

    def set_tile(self, waves: int, rows: int, depth: int = 2, steps: int = 1):
        _check(lib().lbm_batch_set_tile(self.b, int(waves), int(rows), int(depth), int(steps)),
               "lbm_batch_set_tile")

    def get_tile(self):
        w, r, d, k = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
        _check(lib().lbm_batch_get_tile(self.b, C.byref(w), C.byref(r), C.byref(d), C.byref(k)),
               "lbm_batch_get_tile")
        return w.value, r.value, d.value, k.value

    def set_graph_steps(self, k: int):
        _check(lib().lbm_batch_set_graph_steps(self.b, int(k)), "lbm_batch_set_graph_steps")

    def set_mrt(self, rates=None):
        """MRT collision for every run: rates = (s_e, s_eps, s_q) for all runs, or
        one such triple per run; None restores BGK."""
        if rates is None:
            _check(lib().lbm_batch_set_mrt(self.b, None), "lbm_batch_set_mrt")
            return
        r = np.asarray(rates, dtype=np.float64)
        if r.ndim == 1:
            r = np.tile(r, (len(self.ps), 1))
        r = np.ascontiguousarray(r.reshape(len(self.ps), 3))
        _check(lib().lbm_batch_set_mrt(self.b, r.ctypes.data), "lbm_batch_set_mrt")

    def graph_captures(self) -> int:
        n = C.c_int64()
        _check(lib().lbm_batch_graph_captures(self.b, C.byref(n)), "lbm_batch_graph_captures")
        return n.value

    def nodes(self) -> int:
        n = C.c_int64()
        _check(lib().lbm_batch_nodes(self.b, C.byref(n)), "lbm_batch_nodes")
        return n.value

    def close(self):
        if getattr(self, "b", None):
            lib().lbm_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
