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


# ---- capacitance-style systems ---------------------------------------------------
# Conductors (axis-aligned bars) in the three-layer medium: two parallel wires in
# the middle layer, a crossing wire above the top interface and a plate below
# the bottom one, each shifted by a seeded offset of at most 0.02 (every face
# stays at least 0.13 from an interface).  (x0, x1, y0, y1, z0, z1, layer)
_CONDUCTORS = (
    (-0.5, 0.5, -0.20, -0.10, -0.55, -0.45, 1),
    (-0.5, 0.5, 0.10, 0.20, -0.55, -0.45, 1),
    (-0.05, 0.05, -0.5, 0.5, 0.15, 0.25, 0),
    (-0.6, 0.6, -0.6, 0.6, -1.35, -1.25, 2),
)


def _rect_self_integral(a, b):
    """int over [-a, a] x [-b, b] of dA / sqrt(x^2 + y^2) (closed form)."""
    r = np.hypot(a, b)
    return 4.0 * (a * np.log((b + r) / a) + b * np.log((a + r) / b))


def capacitance(n: int = 1500, seed: int = 7):
    """Points at the centres of about n rectangular panels covering the conductors'
    surfaces (spacing h = sqrt(total area / n) on every face), with

      diag[i]  the self term of panel i: the potential at its centre of a unit
               charge spread uniformly over it, 1/(4 pi A) int dA / r
      b[i]     1 on conductor 0, 0 elsewhere (the first column of the
               capacitance matrix: conductor 0 at unit potential)
      cond[i]  the conductor of panel i, area[i] its area.

    The system (diag + G) x = b is the collocation form of the first-kind
    integral equation for the surface charge, in the library's normalisation
    (free part 1/(4 pi r))."""
    rng = np.random.default_rng(seed)
    boxes = []
    for (x0, x1, y0, y1, z0, z1, lay) in _CONDUCTORS:
        s = rng.uniform(-0.02, 0.02, 3)
        boxes.append((x0 + s[0], x1 + s[0], y0 + s[1], y1 + s[1], z0 + s[2], z1 + s[2], lay))
    total = 0.0
    for (x0, x1, y0, y1, z0, z1, _) in boxes:
        ex, ey, ez = x1 - x0, y1 - y0, z1 - z0
        total += 2.0 * (ex * ey + ex * ez + ey * ez)
    h = float(np.sqrt(total / n))
    X, Y, Z, LAY, COND, AREA, DIAG = [], [], [], [], [], [], []
    for c, (x0, x1, y0, y1, z0, z1, lay) in enumerate(boxes):
        lo, hi = (x0, y0, z0), (x1, y1, z1)
        for axis in range(3):          # the face's normal axis
            u, v = [a for a in range(3) if a != axis]
            nu = max(1, int(round((hi[u] - lo[u]) / h)))
            nv = max(1, int(round((hi[v] - lo[v]) / h)))
            du, dv = (hi[u] - lo[u]) / nu, (hi[v] - lo[v]) / nv
            cu = lo[u] + (np.arange(nu) + 0.5) * du
            cv = lo[v] + (np.arange(nv) + 0.5) * dv
            gu, gv = np.meshgrid(cu, cv, indexing="ij")
            self_term = _rect_self_integral(du / 2, dv / 2) / (4.0 * np.pi * du * dv)
            for side in (lo[axis], hi[axis]):
                P = np.zeros((3, gu.size))
                P[axis] = side
                P[u] = gu.ravel()
                P[v] = gv.ravel()
                X.append(P[0]); Y.append(P[1]); Z.append(P[2])
                LAY.append(np.full(gu.size, lay, np.int32))
                COND.append(np.full(gu.size, c, np.int32))
                AREA.append(np.full(gu.size, du * dv))
                DIAG.append(np.full(gu.size, self_term))
    cond = np.concatenate(COND)
    return dict(d=list(THREE_LAYER_D), eps=list(THREE_LAYER_EPS), x=np.concatenate(X), y=np.concatenate(Y),
                z=np.concatenate(Z), layer=np.concatenate(LAY), cond=cond, area=np.concatenate(AREA),
                diag=np.concatenate(DIAG), b=(cond == 0).astype(np.float64), h=h,
                name=f"capacitance: 4 conductors in the 3-layer medium, {len(cond)} panels")
