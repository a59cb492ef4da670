"""Pins of the oracle's surrogate network (oracle/mlp.py), CPU only.

The gradient is pinned by central finite differences of the loss (a check of
the chain rule against the definition of the derivative), the forward pass by
closed forms that a dropped term, a wrong index or a transposed weight breaks.
"""
import numpy as np
import pytest

from oracle import mlp


def _setup(ncomp=5, nout=7, B=9, seed=0, scale=0.3):
    rng = np.random.default_rng(seed)
    lay = mlp.layout(ncomp, nout)
    theta = rng.normal(0.0, scale, lay["total"])
    comp = rng.integers(0, ncomp, B)
    feat = rng.uniform(-1, 1, (B, mlp.F))
    y = rng.normal(0.0, 0.5, (B, nout))
    return lay, theta, comp, feat, y


def test_layout_sizes():
    lay = mlp.layout(100, 41)
    H = mlp.H
    assert lay["total"] == 100 * H + 4 * H + H + 2 * (H * H + H) + H * 41 + 41
    assert lay["E"][0] == 0 and lay["b4"][0] + 41 == lay["total"]


@pytest.mark.parametrize("block", ["E", "A", "b1", "W2", "b2", "W3", "b3", "W4", "b4"])
def test_gradient_matches_finite_differences(block):
    ncomp, nout = 5, 7
    lay, theta, comp, feat, y = _setup(ncomp, nout)
    _, g = mlp.loss_and_grad(theta, ncomp, nout, comp, feat, y)
    off, shp = lay[block]
    size = int(np.prod(shp))
    rng = np.random.default_rng(1)
    idx = off + rng.choice(size, min(size, 12), replace=False)
    if block == "E":  # make sure rows of components present in the batch are probed
        idx = np.concatenate([idx, off + comp[0] * mlp.H + np.arange(3)])
    h = 1e-6
    for i in idx:
        tp = theta.copy()
        tm = theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (mlp.loss(tp, ncomp, nout, comp, feat, y) - mlp.loss(tm, ncomp, nout, comp, feat, y)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(fd)), (block, i, fd, g[i])


def test_unused_component_rows_have_zero_gradient():
    ncomp, nout = 6, 3
    lay, theta, comp, feat, y = _setup(ncomp, nout)
    comp[:] = 2
    _, g = mlp.loss_and_grad(theta, ncomp, nout, comp, feat, y)
    E = g[:ncomp * mlp.H].reshape(ncomp, mlp.H)
    assert np.all(E[[0, 1, 3, 4, 5]] == 0) and np.any(E[2] != 0)


def test_output_closed_form_with_zero_hidden_weights():
    """W2 = W3 = 0: h3 = tanh(b3) for every sample, so out = tanh(b3) W4 + b4."""
    ncomp, nout = 4, 5
    lay, theta, comp, feat, y = _setup(ncomp, nout)
    P = mlp.unpack(theta, lay)
    P["W2"][:] = 0.0
    P["W3"][:] = 0.0
    out, (h1, h2, h3) = mlp.forward(theta, ncomp, nout, comp, feat)
    want = np.tanh(P["b3"]) @ P["W4"] + P["b4"]
    np.testing.assert_allclose(out, np.broadcast_to(want, out.shape), rtol=0, atol=1e-15)
    # first layer: one-hot row + features
    s = 3
    z1 = P["E"][comp[s]] + feat[s] @ P["A"] + P["b1"]
    np.testing.assert_allclose(h1[s], np.tanh(z1), rtol=0, atol=1e-15)


def test_output_layer_is_affine():
    ncomp, nout = 3, 4
    lay, theta, comp, feat, y = _setup(ncomp, nout)
    off, shp = lay["W4"]
    out0, (_, _, h3) = mlp.forward(theta, ncomp, nout, comp, feat)
    t2 = theta.copy()
    t2[off + 5 * nout + 2] += 1.0  # W4[5, 2]
    out1, _ = mlp.forward(t2, ncomp, nout, comp, feat)
    d = out1 - out0
    np.testing.assert_allclose(d[:, 2], h3[:, 5], atol=1e-14)
    assert np.all(d[:, [0, 1, 3]] == 0)


def test_adam_first_step_has_size_lr():
    rng = np.random.default_rng(3)
    th = rng.normal(size=50)
    g = rng.normal(size=50)
    t1, m, v = mlp.adam_step(th, g, np.zeros(50), np.zeros(50), 1, 1e-3, eps=0.0)
    np.testing.assert_allclose(th - t1, 1e-3 * np.sign(g), rtol=1e-12)


def test_adam_constant_gradient_moves_lr_every_step():
    """With the same gradient g at every step, the bias-corrected moments are exactly
    m_t / (1 - beta1^t) = g and v_t / (1 - beta2^t) = g^2 for every t (both geometric
    sums telescope), so each step moves every parameter by lr * sign(g) (eps = 0).
    Without the correction, or with t frozen at 1, step 2 would move 4.25 lr or 1.34 lr."""
    rng = np.random.default_rng(11)
    th = rng.normal(size=40)
    g = rng.normal(size=40)
    m = np.zeros(40)
    v = np.zeros(40)
    cur = th.copy()
    for t in range(1, 6):
        nxt, m, v = mlp.adam_step(cur, g, m, v, t, 1e-3, eps=0.0)
        np.testing.assert_allclose(cur - nxt, 1e-3 * np.sign(g), rtol=1e-10)
        cur = nxt


def test_adam_alternating_gradient_second_step():
    """Gradients g then -g (worked by hand): m_2 = 0.9 (0.1 g) - 0.1 g = -0.01 g,
    v_2 = 0.999 (0.001 g^2) + 0.001 g^2 = 0.001999 g^2; the corrections divide by
    1 - 0.81 = 0.19 and 1 - 0.998001 = 0.001999, so the second step is
    -lr (-0.01 / 0.19) sign(g) = +lr sign(g) / 19."""
    g = np.array([2.0, -0.5, 1e-3])
    th = np.array([0.3, -0.2, 0.1])
    lr = 1e-2
    t1, m, v = mlp.adam_step(th, g, np.zeros(3), np.zeros(3), 1, lr, eps=0.0)
    t2, m, v = mlp.adam_step(t1, -g, m, v, 2, lr, eps=0.0)
    np.testing.assert_allclose(m, -0.01 * g, rtol=1e-12)
    np.testing.assert_allclose(v, 0.001999 * g * g, rtol=1e-12)
    np.testing.assert_allclose(t2 - t1, lr * np.sign(g) / 19.0, rtol=1e-10)


def test_adam_third_step_after_one_kick():
    """Gradients g, 0, 0 (worked by hand): m_3 = 0.81 (0.1 g) = 0.081 g,
    v_3 = 0.998001 (0.001 g^2); corrected: 0.081 / 0.271 g and
    0.000998001 / 0.002997001 g^2, so step 3 is lr * 0.2988929889 / 0.5770614256 sign(g)."""
    g = np.array([3.0, -0.25])
    th = np.array([1.0, 1.0])
    lr = 1e-3
    m = np.zeros(2)
    v = np.zeros(2)
    cur = th
    for t, gt in ((1, g), (2, 0 * g), (3, 0 * g)):
        nxt, m, v = mlp.adam_step(cur, gt, m, v, t, lr, eps=0.0)
        if t < 3:
            cur = nxt
    mh = 0.081 / 0.271
    vh = 0.000998001 / 0.002997001
    np.testing.assert_allclose(cur - nxt, lr * mh / np.sqrt(vh) * np.sign(g), rtol=1e-9)
    np.testing.assert_allclose(mh / np.sqrt(vh), 0.2988929889 / 0.5770614256, rtol=1e-9)
