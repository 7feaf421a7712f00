"""Host logic of the stability sweep (no GPU): the T_min rule and the run set."""
import numpy as np

from paper_1204_4098_amd import lbm, stability as S


def test_lowest_stable_rule():
    grid = [0.5, 0.6, 0.7, 0.8, 0.9]
    assert S.lowest_stable(grid, [0, 0, 1, 1, 1]) == (0.7, True)
    assert S.lowest_stable(grid, [1, 1, 1, 1, 1]) == (0.5, True)
    assert S.lowest_stable(grid, [0, 0, 0, 0, 0]) == (None, True)
    assert S.lowest_stable(grid, [0, 0, 0, 0, 1]) == (0.9, True)
    # a stable island below an unstable temperature is reported as non-monotone
    assert S.lowest_stable(grid, [1, 0, 1, 1, 1]) == (0.7, False)
    # grid order does not matter
    assert S.lowest_stable(grid[::-1], [1, 1, 1, 0, 0]) == (0.7, True)


def test_droplet_runs_follow_the_experiment():
    cases = [S.Case(lbm.LBM_SCHEME_EDM, 0.6), S.Case(lbm.LBM_SCHEME_IMPROVED, 0.7, 0.105)]
    ps, rhos, keys = S.droplet_runs(cases, [0.7, 0.8], nx=40, ny=40, r0=8.0)
    assert len(ps) == len(rhos) == len(keys) == 4
    Tc = S.critical_T()
    for p, r, (case, t) in zip(ps, rhos, keys):
        assert p.scheme == case.scheme and p.tau == case.tau and p.sigma == case.sigma
        assert abs(p.T / Tc - t) < 1e-15
        rl, rg, _ = lbm.lbm_maxwell(lbm.LBM_EOS_CS, 1.0, 4.0, 1.0, 0.0, p.T)
        # Eq. (24): liquid inside, vapour at the corners, midpoint at r = r0
        assert abs(r[20, 20] - rl) < 1e-6 * rl and abs(r[0, 0] - rg) < 1e-9
        assert abs(r[20, 28] - 0.5 * (rl + rg)) < 1e-12
    assert [c.name for c in cases] == ["EDM, tau=0.6", "improved sigma=0.105, tau=0.7"]
