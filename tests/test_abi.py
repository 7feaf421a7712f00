"""The C-ABI library: it builds, loads, exports every symbol include/*.h declares,
and its host-only thermodynamics agrees with the oracle (no GPU needed)."""
import glob
import math
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = []
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        txt = open(h).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        names += re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*(lbm_[a-z0-9_]+|mlp_[a-z0-9_]+)\s*\(",
                            txt, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def L():
    from paper_1204_4098_amd import lbm
    if not os.path.exists(lbm.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return lbm


def test_header_declares_the_boundary():
    names = _declared()
    for required in ("lbm_init", "lbm_step", "lbm_moments", "lbm_batch_init", "lbm_batch_step",
                     "lbm_batch_coexistence", "lbm_destroy"):
        assert required in names


def test_library_exports_every_declared_symbol(L):
    import ctypes
    so = ctypes.CDLL(L.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(so, n)]
    assert not missing, missing


def test_strerror_and_invalid_params(L):
    assert L.lbm_strerror(L.LBM_EDIVERGED) == "the run diverged"
    p = L.params(64, 32, tau=0.5, T=0.08)
    with pytest.raises(L.LbmError):
        L.lbm_workspace_bytes(p)
    p = L.params(2, 32, T=0.08)
    with pytest.raises(L.LbmError):
        L.lbm_workspace_bytes(p)
    for scheme in (-1, 5):
        with pytest.raises(L.LbmError):
            L.lbm_workspace_bytes(L.params(64, 32, T=0.08, scheme=scheme))
    for scheme in range(5):
        assert L.lbm_workspace_bytes(L.params(64, 32, T=0.08, scheme=scheme)) > 0
    assert L.lbm_workspace_bytes(L.params(64, 32, T=0.08)) >= 2 * 9 * 64 * 32 * 8


def test_critical_points_match_oracle(L):
    from oracle import thermo as th
    Tc, rc = L.lbm_critical_point(L.LBM_EOS_CS, 1.0, 4.0, 1.0, 0.0)
    oTc, orc = th.critical_cs()
    assert abs(Tc / oTc - 1) < 1e-12 and abs(rc / orc - 1) < 1e-9
    Tc, rc = L.lbm_critical_point(L.LBM_EOS_PR, 2 / 49, 2 / 21, 1.0, 0.344)
    oTc, orc = th.critical_pr()
    assert abs(Tc / oTc - 1) < 1e-12 and abs(rc / orc - 1) < 1e-9


@pytest.mark.parametrize("t", [0.55, 0.7, 0.8, 0.95])
def test_maxwell_matches_oracle_cs(L, t):
    from oracle import thermo as th
    Tc, _ = L.lbm_critical_point(L.LBM_EOS_CS, 1.0, 4.0, 1.0, 0.0)
    rl, rg, p0 = L.lbm_maxwell(L.LBM_EOS_CS, 1.0, 4.0, 1.0, 0.0, t * Tc)
    m = th.maxwell_cs(t)
    assert abs(rl / m.rho_l - 1) < 1e-10 and abs(rg / m.rho_g - 1) < 1e-9


@pytest.mark.parametrize("t", [0.6, 0.8])
def test_maxwell_matches_oracle_pr(L, t):
    from oracle import thermo as th
    Tc, _ = L.lbm_critical_point(L.LBM_EOS_PR, 2 / 49, 2 / 21, 1.0, 0.344)
    rl, rg, p0 = L.lbm_maxwell(L.LBM_EOS_PR, 2 / 49, 2 / 21, 1.0, 0.344, t * Tc)
    m = th.maxwell_pr(t)
    assert abs(rl / m.rho_l - 1) < 1e-10 and abs(rg / m.rho_g - 1) < 1e-9


def test_pressure_matches_oracle(L):
    from oracle import lbm as olbm
    from oracle import thermo as th
    Tc, _ = th.critical_pr()
    p = L.params(8, 8, eos=L.LBM_EOS_PR, a=2 / 49, b=2 / 21, R=1.0, omega=0.344, T=0.6 * Tc)
    op = olbm.Params(nx=8, ny=8, eos=olbm.EOS_PR, a=2 / 49, b=2 / 21, R=1.0, omega=0.344, T=0.6 * Tc, Tc=Tc)
    for rho in (0.01, 1.0, 8.0):
        assert abs(L.lbm_pressure(p, rho) - olbm.p_eos(op, rho)) < 1e-13 * max(1, abs(olbm.p_eos(op, rho)))
