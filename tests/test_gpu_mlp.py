"""The surrogate network's HIP kernels (through the C ABI) against the FP64 oracle."""
import numpy as np
import pytest

import synth
from oracle import mlp as omlp

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def M():
    import torch
    from paper_1204_4098_amd import mlp
    assert torch.cuda.is_available()
    return mlp


def _data(B, seed=4):
    rng = np.random.default_rng(seed)
    X = np.column_stack([rng.uniform(0.5, 0.95, B), rng.uniform(0.6, 1.5, B),
                         rng.uniform(0, 0.2, B)]).astype(np.float32)
    # a smooth synthetic map with the shape of coexistence curves
    t, tau, s = X[:, 0].astype(np.float64), X[:, 1].astype(np.float64), X[:, 2].astype(np.float64)
    T = np.column_stack([np.log(0.2 + 0.4 * (1 - t) ** 0.5 + 0.01 * s),
                         np.log(0.09 * np.exp(-6 * (1 - t)) * (1 + 2 * s) * (1 + 0.01 * tau))]).astype(np.float32)
    return X, T


def _norm(M, X, T):
    n = omlp.norm_from(X.astype(np.float64), T.astype(np.float64))
    f32 = {k: np.asarray(v, dtype=np.float32).astype(np.float64) for k, v in n.items()}
    return M.make_norm(n["in_mean"], n["in_std"], n["out_mean"], n["out_std"]), f32


def _params(seed=1):
    th = synth.mlp_init(seed)
    rng = np.random.default_rng(seed)
    return (th + (0.05 * rng.standard_normal(th.size)).astype(np.float32)).astype(np.float32)


@pytest.mark.parametrize("B", [1, 31, 1000, 4096])
def test_forward_matches_oracle(M, B):
    X, T = _data(B)
    nrm, n64 = _norm(M, X, T)
    th = _params()
    net = M.Mlp(th, nrm, max_batch=B)
    y = net.forward(X)
    ref = omlp.predict(th.astype(np.float64), X.astype(np.float64), n64, emulate_bf16=True)
    err = np.abs(y - ref) / np.maximum(np.abs(ref), 1e-3)
    # bfloat16 rounding decisions of hidden activations can differ where FP32 and
    # FP64 pre-activations straddle a rounding boundary: allow rare, small outliers
    assert np.quantile(err, 0.99) < 2e-5, np.quantile(err, 0.99)
    assert err.max() < 5e-3, err.max()
    net.close()


def test_gradient_matches_oracle(M):
    B = 2000
    X, T = _data(B, seed=7)
    nrm, n64 = _norm(M, X, T)
    th = _params(3)
    net = M.Mlp(th, nrm, max_batch=B)
    loss, g = net.gradient(X, T)
    rl, rg = omlp.loss_and_grad(th.astype(np.float64), X.astype(np.float64), T.astype(np.float64), n64)
    assert abs(loss / rl - 1) < 1e-4
    # element by element, each entry against the largest entry of its block.  The
    # kernels accumulate in FP32 and round FP32 (not FP64) pre-activations and
    # errors to bfloat16, so a product whose operand straddles a bfloat16 rounding
    # boundary can differ by one bfloat16 ulp (2^-8 relative) from the oracle's.
    # Measured on MI355X: block maxima 1.6e-7 .. 7.6e-6 and no entry above 2e-5;
    # the bound allows 1 % of a block above 2e-5 (rounding-boundary outliers)
    # and none above 1e-4.
    for name, shape in omlp.SHAPES:
        a = omlp.unpack(g)[name]
        b = omlp.unpack(rg)[name]
        err = np.abs(a - b) / np.abs(b).max()
        out = int(np.sum(err > 2e-5))
        print(f"{name}: max {err.max():.2e}, p99 {np.quantile(err, 0.99):.2e}, "
              f"median {np.median(err):.2e}, {out} of {err.size} above 2e-5", flush=True)
        assert err.max() < 1e-4, (name, err.max())
        assert out <= err.size // 100, (name, out)
    # deterministic: the same call gives the same bits
    loss2, g2 = net.gradient(X, T)
    assert loss2 == loss and np.array_equal(g, g2)
    net.close()


def test_adam_step_matches_oracle(M):
    X, T = _data(64)
    nrm, _ = _norm(M, X, T)
    th = _params(5)
    net = M.Mlp(th, nrm, max_batch=64)
    rng = np.random.default_rng(2)
    g1 = (1e-2 * rng.standard_normal(th.size)).astype(np.float32)
    g2 = (1e-2 * rng.standard_normal(th.size)).astype(np.float32)
    net.adam(g1, 1e-3)
    net.adam(g2, 1e-3)
    p = th.astype(np.float64); m = np.zeros_like(p); v = np.zeros_like(p)
    p, m, v = omlp.adam(p, m, v, g1.astype(np.float64), 1)
    p, m, v = omlp.adam(p, m, v, g2.astype(np.float64), 2)
    assert np.max(np.abs(net.params() - p)) < 1e-6
    net.close()


def test_training_fits_smooth_map(M):
    X, T = _data(8192, seed=11)
    nrm, n64 = _norm(M, X, T)
    net = M.Mlp(synth.mlp_init(), nrm, max_batch=1024)
    hist = net.train(X, T, steps=3000, lr=2e-3, batch=1024, log_every=500)
    assert hist[-1][1] < 0.02 * hist[0][1], hist
    Xv, Tv = _data(512, seed=12)
    rms = np.sqrt(np.mean((net.forward(Xv) - Tv) ** 2, axis=0))
    assert np.all(rms < 0.02), rms
    net.close()
