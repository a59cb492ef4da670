"""Seeded synthetic workloads for the layered-media FMM.

This module only draws inputs (positions, layer ids, charges); it holds none
of the method's arithmetic and is shared by the tests, the benchmark and the
CPU oracle's callers.  The paper's own test geometry (Sec. 4: charges in
irregular axisymmetric domains) is replaced by boxes with a 0.1 margin to every
interface; the layered media and sizes follow the five workloads below.

Common recipe (x, y ~ U[-0.5, 0.5]; q ~ U[-1, 1]):
  top layer    z ~ U(d_0 + 0.1, d_0 + 1.1)
  finite layer z ~ U(d_l + 0.1, d_{l-1} - 0.1)
  bottom layer z ~ U(d_{L-1} - 1.1, d_{L-1} - 0.1)
"""
from __future__ import annotations

import numpy as np

THREE_LAYER_D = (0.0, -1.0)
THREE_LAYER_EPS = (1.0, 5.0, 2.0)


def layer_zrange(d, layer):
    L = len(d)
    if layer == 0:
        return d[0] + 0.1, d[0] + 1.1
    if layer == L:
        return d[L - 1] - 1.1, d[L - 1] - 0.1
    return d[layer] + 0.1, d[layer - 1] - 0.1


def split_even(n, nlayers):
    base = n // nlayers
    counts = [base] * nlayers
    for i in range(n - base * nlayers):
        counts[i] += 1
    return counts


def _uniform_layer(rng, d, layer, count):
    z0, z1 = layer_zrange(d, layer)
    x = rng.uniform(-0.5, 0.5, count)
    y = rng.uniform(-0.5, 0.5, count)
    z = rng.uniform(z0, z1, count)
    return x, y, z


def _gaussian_mixture_layer(rng, d, layer, count, ncomp=8, sd=0.05):
    z0, z1 = layer_zrange(d, layer)
    lo = np.array([-0.5, -0.5, z0])
    hi = np.array([0.5, 0.5, z1])
    centers = rng.uniform(lo, hi, size=(ncomp, 3))
    comp = rng.integers(0, ncomp, count)
    pts = centers[comp] + rng.normal(0.0, sd, size=(count, 3))
    bad = np.any((pts <= lo) | (pts >= hi), axis=1)
    while bad.any():
        nb = int(bad.sum())
        pts[bad] = centers[comp[bad]] + rng.normal(0.0, sd, size=(nb, 3))
        bad = np.any((pts <= lo) | (pts >= hi), axis=1)
    return pts[:, 0].copy(), pts[:, 1].copy(), pts[:, 2].copy()


def make_layered(d, eps, counts, seed, nrhs=1, clustered_layers=()):
    """Points layer by layer (top first), then charges [nrhs, N]."""
    rng = np.random.default_rng(seed)
    xs, ys, zs, ls = [], [], [], []
    for layer, c in enumerate(counts):
        if layer in clustered_layers:
            x, y, z = _gaussian_mixture_layer(rng, d, layer, c)
        else:
            x, y, z = _uniform_layer(rng, d, layer, c)
        xs.append(x)
        ys.append(y)
        zs.append(z)
        ls.append(np.full(c, layer, dtype=np.int32))
    x = np.concatenate(xs)
    y = np.concatenate(ys)
    z = np.concatenate(zs)
    layer = np.concatenate(ls)
    q = rng.uniform(-1.0, 1.0, size=(nrhs, len(x)))
    return dict(d=np.asarray(d, np.float64), eps=np.asarray(eps, np.float64),
                x=x, y=y, z=z, layer=layer, q=q)


def config(idx: int, n: int | None = None, seed: int | None = None):
    """Workload idx in 0..4 (see the table in the design notes); n overrides the size."""
    if idx == 0:
        N = n or 1200
        w = make_layered(THREE_LAYER_D, THREE_LAYER_EPS, split_even(N, 3), seed or 1)
        w.update(name="3-layer N=1200 uniform p=8", p=8, leaf_cap=40)
    elif idx == 1:
        N = n or 262144
        w = make_layered(THREE_LAYER_D, THREE_LAYER_EPS, split_even(N, 3), seed or 2,
                         clustered_layers=(1,))
        w.update(name="3-layer N=262144 clustered middle p=10/12", p=10, leaf_cap=64)
    elif idx == 2:
        N = n or 1048576
        w = make_layered(THREE_LAYER_D, THREE_LAYER_EPS, split_even(N, 3), seed or 3)
        w.update(name="3-layer N=1048576 uniform p=10", p=10, leaf_cap=64)
    elif idx == 3:
        N = n or 524288
        w = make_layered((0.0, -0.6, -1.4), (1.0, 3.9, 11.7, 2.5), split_even(N, 4),
                         seed or 4, nrhs=64)
        w.update(name="4-layer N=524288 uniform 64 rhs p=10", p=10, leaf_cap=64)
    elif idx == 4:
        N = n or 2097152
        rng = np.random.default_rng(5)
        d = (0.0, -0.5, -1.0, -1.8, -2.6)
        eps = rng.uniform(1.0, 12.0, 6)
        wts = 10.0 ** rng.uniform(0.0, 2.0, 6)
        raw = N * wts / wts.sum()
        counts = np.floor(raw).astype(int)
        rem = N - counts.sum()
        order = np.argsort(-(raw - counts), kind="stable")
        counts[order[:rem]] += 1
        w = make_layered(d, eps, [int(c) for c in counts], seed or 5)
        w.update(name="6-region N=2097152 log-uniform p=10", p=10, leaf_cap=64)
    else:
        raise ValueError(idx)
    return w
