"""Pins of the warm-start network oracle: gradients against central finite
differences, the known first step of Adam, and a fit on a learnable map."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import mlp as N
from paper_2009_02845_amd import synth


def _batch(B=7, d=12, k=4, H=9, seed=0, density=0.3):
    g = np.random.default_rng(seed)
    p = {k_: v.astype(np.float64) for k_, v in synth.mlp_init(d, k, H, seed).items()}
    p["b1"] = g.standard_normal(H) * 0.3
    p["b2"] = g.standard_normal(k) * 0.3 + 0.5
    A = sp.random(B, d, density=density, format="csr", random_state=seed) * 3.0
    U = g.random((B, k))
    Y = g.random((B, k))
    return p, A, U, Y


@pytest.mark.parametrize("residual", [False, True])
def test_gradients_match_central_differences(residual):
    p, A, U, Y = _batch()
    Hpre, _, Ypre, _ = N.forward(p, A, U, residual)
    # keep away from the ReLU kinks so the loss is smooth at p
    assert np.min(np.abs(Hpre)) > 1e-4 and np.min(np.abs(Ypre)) > 1e-4
    g, L = N.backward(p, A, U, Y, residual)
    h = 1e-6
    for name in N.PARAMS:
        num = np.zeros_like(p[name])
        it = np.nditer(p[name], flags=["multi_index"])
        for _ in it:
            idx = it.multi_index
            q = {k_: v.copy() for k_, v in p.items()}
            q[name][idx] += h
            lp = N.loss(N.forward(q, A, U, residual)[3], Y)
            q[name][idx] -= 2 * h
            lm = N.loss(N.forward(q, A, U, residual)[3], Y)
            num[idx] = (lp - lm) / (2 * h)
        err = np.linalg.norm(num - g[name]) / max(np.linalg.norm(num), 1e-12)
        assert err < 1e-6, (name, err)


def test_adam_first_step_is_signed_lr():
    # with zero moments, the bias-corrected first step is lr * g / (|g| + eps)
    p, A, U, Y = _batch(seed=1)
    g, _ = N.backward(p, A, U, Y)
    m = {k_: np.zeros_like(v) for k_, v in p.items()}
    v = {k_: np.zeros_like(x) for k_, x in p.items()}
    old = {k_: x.copy() for k_, x in p.items()}
    N.adam_step(p, g, m, v, 1, lr=1e-3)
    for name in N.PARAMS:
        big = np.abs(g[name]) > 1e-4
        assert np.allclose((old[name] - p[name])[big], 1e-3 * np.sign(g[name][big]), rtol=1e-3, atol=0)


@pytest.mark.parametrize("residual", [False, True])
def test_training_fits_a_learnable_map(residual):
    # target: y = relu(u + 0.5 * a[:, :k]) -- a two-layer ReLU net can fit it
    g = np.random.default_rng(2)
    B, d, k, H = 256, 10, 4, 32
    A = sp.csr_matrix(g.random((B, d)) * (g.random((B, d)) < 0.5))
    U = g.random((B, k))
    Y = np.maximum(U + 0.5 * A.toarray()[:, :k], 0.0)
    p = {k_: v.astype(np.float64) for k_, v in synth.mlp_init(d, k, H, 3).items()}
    m = {k_: np.zeros_like(v) for k_, v in p.items()}
    v = {k_: np.zeros_like(x) for k_, x in p.items()}
    first = N.loss(N.forward(p, A, U, residual)[3], Y)
    for t in range(1, 1501):
        gr, _ = N.backward(p, A, U, Y, residual)
        N.adam_step(p, gr, m, v, t, lr=3e-3)
    last = N.loss(N.forward(p, A, U, residual)[3], Y)
    assert last < 0.02 * first


def test_residual_variant_adds_the_input_row():
    # the two forms differ exactly by u in the output pre-activation
    p, A, U, _ = _batch(seed=4)
    plain = N.forward(p, A, U, residual=False)
    res = N.forward(p, A, U, residual=True)
    assert np.allclose(res[2] - plain[2], U, rtol=0, atol=1e-15)
    assert np.array_equal(res[1], plain[1])
