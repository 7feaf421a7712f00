"""The learned sigma proposal, end to end on the GPU at the configured scale:
10,240 batched flat-interface runs of 30,000 steps -> network trained by the
library's kernels (80/20 split) -> proposed sigma for 32 held-out (T/Tc, tau)
pairs -> FP64 256 x 32 lattice verification of 30,000 steps, compared with the
method without the network (the paper's fixed sigma = 0.105, the theory sigma*,
LB bisection)."""
import json
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden", "sigma_star_cs.json")


@pytest.fixture(scope="module")
def S():
    import torch
    from paper_1204_4098_amd import surrogate
    assert torch.cuda.is_available()
    return surrogate


@pytest.fixture(scope="module")
def trained(S):
    X, Y, info = S.dataset(10240, steps=30000, batch=256, log=print)
    print("dataset", info, X.shape)
    assert X.shape[0] >= 8000, info
    net, rep = S.fit(X, Y, steps=120000, lr=2e-3, batch=1024)
    print("surrogate fit:", {k: v for k, v in rep.items() if k != "loss_history"})
    # held-out runs span rho_g over three decades (T/Tc 0.5 .. 0.95): median error within
    # 1 % (measured 0.035 % for rho_l, 0.27 % for rho_g); the lattice verification decides
    assert max(rep["heldout_rel_err_median"]) < 0.01, rep
    return net


def test_surrogate_gains_over_fixed_and_theory_sigma(S, trained):
    pairs = S.heldout_pairs(32)
    g = json.load(open(GOLD))
    theory = [float(np.interp(t, g["t_over_tc"], g["sigma_star"])) for t, _ in pairs]
    sig, e_net, runs = S.propose_and_verify(trained, pairs, steps=30000, tol=0.01, bisect_iters=8)
    e_fix, _ = S.verify(pairs, [0.105] * len(pairs), steps=30000)
    e_th, _ = S.verify(pairs, theory, steps=30000)
    worst = lambda e: np.max(e, axis=1)
    print("pairs", [(round(a, 3), round(b, 3)) for a, b in pairs])
    print("sigma: net", np.round(sig, 4), "theory", np.round(theory, 4), "lattice runs", runs)
    print("max(|drho_l|,|drho_g|)/rho: net", np.round(worst(e_net), 4), "fixed 0.105",
          np.round(worst(e_fix), 4), "theory", np.round(worst(e_th), 4))
    assert np.all(worst(e_net) <= 0.01)                 # every pick verified within 1 %
    # the network's own first pick lands within 1 % (measured: every one of the 32; a
    # Newton step with the network's slope, then LB bisection, would settle a miss)
    print("first picks within 1 %:", int(np.sum(runs == 1)), "of", len(pairs))
    assert np.sum(runs == 1) >= 30, runs
    assert np.mean(worst(e_net)) < np.mean(worst(e_fix))
    assert np.mean(worst(e_net)) < np.mean(worst(e_th))
    # cheaper than bisection: at most two lattice runs per pair on average
    assert runs.mean() <= 2.0, runs


def test_bisection_baseline(S):
    pairs = S.heldout_pairs(4, seed=99)
    sig_b, nruns_b = S.bisect_sigma(pairs, steps=30000, iters=8)
    e_b, _ = S.verify(pairs, sig_b, steps=30000)
    print("bisection sigma", np.round(sig_b, 4), "errors", np.round(np.max(e_b, 1), 4))
    assert nruns_b == 8 * len(pairs)
    assert np.all(np.max(e_b, 1) < 0.01)
