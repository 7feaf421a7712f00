"""lbm_mass_noalloc (static device scratch, no allocation) against lbm_mass,
through the C ABI, on two calls in a row, the second with a smaller input."""
import ctypes as C

import numpy as np
import pytest

from tests.gpu_common import CS, pair, slab_rho, droplet_rho

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import torch
    from paper_1204_4098_amd import lbm
    assert torch.cuda.is_available()
    lbm.lib()
    return lbm


def _noalloc(L, lat):
    b0, b1, cur = lat.device_buffers()
    fixed = (C.c_int64 * 2)()
    m = C.c_double()
    p = lat.p
    st = L.lib().lbm_mass_noalloc(b1 if cur else b0, p.nx, p.ny, p.precision, lat.rho_ref(),
                                  lat.stream.cuda_stream, fixed, C.byref(m))
    assert st == L.LBM_OK, L.lbm_strerror(st)
    return m.value, (fixed[1] << 64) + (fixed[0] & ((1 << 64) - 1))


def test_noalloc_mass_equals_lbm_mass_twice(L):
    # a large FP32-deviation droplet lattice, then a smaller FP64 slab: both bit for bit
    cases = [(pair(L, 700, 300, t=0.8, precision=1)[0], droplet_rho(700, 300, CS, 0.8, 60), 37),
             (pair(L, 64, 32, t=0.8, precision=0)[0], slab_rho(64, 32, CS, 0.8), 11)]
    for gp, rho0, steps in cases:
        lat = L.Lattice(gp, rho0)
        lat.step(steps)
        ref = lat.mass()
        got = _noalloc(L, lat)
        assert got[1] == ref[1]
        assert got[0] == ref[0]            # same partials, same summation order
        lat.close()


def test_noalloc_rejects_bad_sizes(L):
    fixed = (C.c_int64 * 2)()
    m = C.c_double()
    lib = L.lib()
    dummy = C.c_void_p(256)   # never dereferenced: every call below is refused on the host
    assert lib.lbm_mass_noalloc(dummy, 65536, 65536, 0, 0.0, None, fixed, C.byref(m)) == L.LBM_ENOSPACE
    assert lib.lbm_mass_noalloc(dummy, 2, 64, 0, 0.0, None, fixed, C.byref(m)) == L.LBM_EINVAL
    assert lib.lbm_mass_noalloc(dummy, 64, 64, 7, 0.0, None, fixed, C.byref(m)) == L.LBM_EINVAL
    assert lib.lbm_mass_noalloc(None, 64, 64, 0, 0.0, None, fixed, C.byref(m)) == L.LBM_EINVAL
