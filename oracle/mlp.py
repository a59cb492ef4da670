"""Oracle -- TEST INFRASTRUCTURE ONLY: the surrogate network in plain numpy, FP64.

The surrogate of the reaction Sommerfeld integrals is a 4-layer perceptron of
width 128 with tanh activations (the learned form of the method: the network
stands in for the 4p+1 initial values of eq. scaledsommerfeldint per
component, with eq. recurrence for the rest).  This module writes out its
definition -- forward pass, mean-squared loss, gradient by the chain rule, and
the Adam update -- with no blocking or fusion, so that the GPU kernels can be
checked against it.  It shares no code with the GPU path.

Parameters, one flat vector, in this order (W[k, j] maps input k to output j):
    E  [ncomp, H]   first layer, one-hot component input (an embedding)
    A  [F, H]       first layer, continuous features
    b1 [H]
    W2 [H, H],  b2 [H]
    W3 [H, H],  b3 [H]
    W4 [H, nout], b4 [nout]
Network, for a sample (c, f):
    h1 = tanh(E[c] + f A + b1);  h2 = tanh(h1 W2 + b2);  h3 = tanh(h2 W3 + b3)
    out = h3 W4 + b4
Loss over a batch of B samples: mean over the B * nout entries of (out - y)^2.

Pins (tests/test_oracle_mlp.py): central finite differences of the loss for
every parameter block, the closed form of the output when the hidden weights
vanish, linearity of the output layer, and Adam's first step (|update| = lr).
"""
from __future__ import annotations

import numpy as np

H = 128
F = 4


def layout(ncomp: int, nout: int) -> dict:
    """Offsets and shapes of the parameter blocks in the flat vector."""
    shapes = [("E", (ncomp, H)), ("A", (F, H)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)),
              ("W3", (H, H)), ("b3", (H,)), ("W4", (H, nout)), ("b4", (nout,))]
    off = 0
    out = {}
    for name, shp in shapes:
        size = int(np.prod(shp))
        out[name] = (off, shp)
        off += size
    out["total"] = off
    return out


def unpack(theta, lay):
    blocks = {k: v for k, v in lay.items() if k != "total"}
    return {k: theta[o:o + int(np.prod(s))].reshape(s) for k, (o, s) in blocks.items()}


def forward(theta, ncomp, nout, comp, feat):
    """Network output [B, nout] and the hidden activations (h1, h2, h3)."""
    P = unpack(np.asarray(theta, np.float64), layout(ncomp, nout))
    f = np.asarray(feat, np.float64)
    h1 = np.tanh(P["E"][comp] + f @ P["A"] + P["b1"])
    h2 = np.tanh(h1 @ P["W2"] + P["b2"])
    h3 = np.tanh(h2 @ P["W3"] + P["b3"])
    out = h3 @ P["W4"] + P["b4"]
    return out, (h1, h2, h3)


def loss(theta, ncomp, nout, comp, feat, y):
    out, _ = forward(theta, ncomp, nout, comp, feat)
    return float(np.mean((out - np.asarray(y, np.float64)) ** 2))


def loss_and_grad(theta, ncomp, nout, comp, feat, y):
    """Loss and its gradient with respect to the flat parameter vector (chain rule)."""
    lay = layout(ncomp, nout)
    P = unpack(np.asarray(theta, np.float64), lay)
    f = np.asarray(feat, np.float64)
    y = np.asarray(y, np.float64)
    out, (h1, h2, h3) = forward(theta, ncomp, nout, comp, feat)
    B = out.shape[0]
    r = out - y
    L = float(np.mean(r ** 2))
    d_out = 2.0 * r / (B * nout)
    g = {}
    g["W4"] = h3.T @ d_out
    g["b4"] = d_out.sum(0)
    d_z3 = (d_out @ P["W4"].T) * (1.0 - h3 ** 2)
    g["W3"] = h2.T @ d_z3
    g["b3"] = d_z3.sum(0)
    d_z2 = (d_z3 @ P["W3"].T) * (1.0 - h2 ** 2)
    g["W2"] = h1.T @ d_z2
    g["b2"] = d_z2.sum(0)
    d_z1 = (d_z2 @ P["W2"].T) * (1.0 - h1 ** 2)
    g["A"] = f.T @ d_z1
    g["b1"] = d_z1.sum(0)
    gE = np.zeros_like(P["E"])
    for s in range(B):
        gE[comp[s]] += d_z1[s]
    g["E"] = gE
    grad = np.zeros(lay["total"])
    for k, v in lay.items():
        if k != "total":
            o, s = v
            grad[o:o + int(np.prod(s))] = g[k].ravel()
    return L, grad


def adam_step(theta, grad, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba, Algorithm 1) at step t >= 1; returns new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad ** 2
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
