"""Host logic of the per-droplet diagnostics (no GPU): region sums on synthetic fields."""
import numpy as np
import pytest

from paper_1204_4098_amd import droplets as D


def _field(nx, ny, centers, radii, inside, outside):
    y, x = np.meshgrid(np.arange(ny, dtype=float), np.arange(nx, dtype=float), indexing="ij")
    f = np.full((ny, nx), outside)
    for (cx, cy), r in zip(centers, radii):
        dx = np.abs(x - cx); dx = np.minimum(dx, nx - dx)
        dy = np.abs(y - cy); dy = np.minimum(dy, ny - dy)
        f[dx * dx + dy * dy <= r * r] = inside
    return f


def test_report_on_step_profiles_with_periodic_wrap():
    nx, ny = 300, 200
    centers = [(150.0, 100.0), (5.0, 190.0)]          # the second wraps around both edges
    radii = [20.0, 12.0]
    rho = _field(nx, ny, centers, radii, 0.4, 0.01)
    p = _field(nx, ny, centers, radii, 2e-3, 1e-3)
    rep = D.report(rho, p, centers, radii)
    assert np.allclose(rep["dp"], 1e-3) and rep["p_far"] == pytest.approx(1e-3)
    for (cx, cy), r, m in zip(centers, radii, rep["mass"]):
        y, x = np.meshgrid(np.arange(ny, dtype=float), np.arange(nx, dtype=float), indexing="ij")
        dx = np.abs(x - cx); dx = np.minimum(dx, nx - dx)
        dy = np.abs(y - cy); dy = np.minimum(dy, ny - dy)
        d2 = dx * dx + dy * dy
        assert m == pytest.approx(rho[d2 <= (r + 8) ** 2].sum(), rel=1e-12)


def test_report_rejects_a_lattice_without_far_vapour():
    rho = np.full((40, 40), 0.3)
    with pytest.raises(ValueError):
        D.report(rho, rho, [(20.0, 20.0)], [15.0])


def test_layout_is_the_workload_layout():
    c, r = D.layout()
    assert len(c) == len(r) == 64 and min(r) >= 40 and max(r) <= 120
