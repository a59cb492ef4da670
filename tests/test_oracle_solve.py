"""Pins of the oracle's dense matrix and dense solve (the reference for the GMRES
solve around the FMM matvec), and of the capacitance-style workload.

* matrix(...) @ q equals the direct sum potential(q) (the pinned pair kernel),
  for the three-layer image series and the four-layer quadrature.
* Reciprocity of the layered Green's function: eps_i G_ij = eps_j G_ji, which
  any transposed or mis-indexed reaction term breaks.
* solve_dense: the product (G + diag) x, formed separately, returns b; the
  conductors' capacitance matrix in physical charge (eps times the library's
  charge, whose free part is q / (4 pi r)), C_ij = eps_c(i) sum_{k in i} x^(j)_k,
  is symmetric and follows the maximum principle (C_jj > 0, C_ij < 0 for
  i != j, sum_i C_ij > 0).
* The workload: panel areas sum to the conductors' surface area, every panel
  is at least 0.13 from an interface, and the panel self term matches the
  closed form for a square (8 a ln(1 + sqrt 2) over a side 2a).
"""
import numpy as np
import pytest

import oracle
from paper_1908_10863_amd import workloads as W


@pytest.fixture(scope="module")
def cap():
    w = W.capacitance(600, seed=7)
    G = oracle.matrix(w["d"], w["eps"], w["x"], w["y"], w["z"], w["layer"], method="image3")
    return w, G


def test_matrix_matches_direct_sum_three_layers(cap):
    w, G = cap
    q = np.random.default_rng(1).normal(size=len(w["x"]))
    phi = oracle.potential(w["d"], w["eps"], w["x"], w["y"], w["z"], w["layer"], q, method="image3")
    assert np.abs(G @ q - phi).max() <= 1e-12 * np.abs(phi).max()


def test_matrix_matches_direct_sum_four_layers_quadrature():
    w = W.config(3, n=32, seed=9)
    G = oracle.matrix(w["d"], w["eps"], w["x"], w["y"], w["z"], w["layer"], method="quad")
    q = np.random.default_rng(2).normal(size=32)
    phi = oracle.potential(w["d"], w["eps"], w["x"], w["y"], w["z"], w["layer"], q, method="quad")
    assert np.abs(G @ q - phi).max() <= 1e-12 * np.abs(phi).max()
    e = np.asarray(w["eps"])[w["layer"]]
    EG = e[:, None] * G
    assert np.abs(EG - EG.T).max() <= 1e-9 * np.abs(EG).max()


def test_reciprocity_three_layers(cap):
    w, G = cap
    e = np.asarray(w["eps"])[w["layer"]]
    EG = e[:, None] * G
    assert np.abs(EG - EG.T).max() <= 1e-13 * np.abs(EG).max()
    # and the unweighted matrix is not symmetric across layers of different eps
    assert np.abs(G - G.T).max() > 1e-3 * np.abs(G).max()


def test_solve_dense_returns_b(cap):
    w, G = cap
    x = oracle.solve_dense(G, w["diag"], w["b"])
    r = w["b"] - (G @ x + w["diag"] * x)
    assert np.linalg.norm(r) <= 1e-12 * np.linalg.norm(w["b"])


def test_capacitance_coefficients(cap):
    w, G = cap
    nc = int(w["cond"].max()) + 1
    C = np.zeros((nc, nc))
    for j in range(nc):
        xj = oracle.solve_dense(G, w["diag"], (w["cond"] == j).astype(np.float64))
        for i in range(nc):
            C[i, j] = xj[w["cond"] == i].sum()
    lay = np.array([w["layer"][w["cond"] == c][0] for c in range(nc)])
    C = np.asarray(w["eps"])[lay][:, None] * C
    assert np.abs(C - C.T).max() <= 1e-10 * np.abs(C).max()
    assert (np.diag(C) > 0).all()
    assert (C[~np.eye(nc, dtype=bool)] < 0).all()
    assert (C.sum(axis=0) > 0).all()


def test_workload_geometry():
    w = W.capacitance(5000, seed=3)
    area = 0.0
    for (x0, x1, y0, y1, z0, z1, _) in W._CONDUCTORS:
        ex, ey, ez = x1 - x0, y1 - y0, z1 - z0
        area += 2 * (ex * ey + ex * ez + ey * ez)
    assert abs(w["area"].sum() - area) <= 1e-12 * area
    d = np.asarray(w["d"])
    assert np.abs(w["z"][:, None] - d[None, :]).min() >= 0.13
    assert set(np.unique(w["b"])) == {0.0, 1.0}
    assert np.array_equal(w["b"], (w["cond"] == 0).astype(float))
    # every point lies in its layer
    zlo = np.array([d[0], d[1], -np.inf])
    zhi = np.array([np.inf, d[0], d[1]])
    assert ((w["z"] > zlo[w["layer"]]) & (w["z"] < zhi[w["layer"]])).all()
    # self term of a square panel of side 2a: 8 a ln(1 + sqrt 2) / (4 pi (2a)^2)
    a = 0.01
    assert abs(W._rect_self_integral(a, a) - 8 * a * np.log(1 + np.sqrt(2))) <= 1e-15


def test_rectangular_panel_self_integral():
    """The closed form of int over [-a, a] x [-b, b] of dA / r for rectangles, against
    adaptive quadrature in polar coordinates about the centre (the integrand's
    singularity cancels against the Jacobian: int dtheta int_0^{R(theta)} dr)."""
    from scipy.integrate import quad
    for a, b in [(0.5, 0.5), (1.0, 0.25), (0.03, 0.7), (2.0, 1.0)]:
        # r runs from 0 to the rectangle's edge along each direction
        def edge(t):
            c, s = abs(np.cos(t)), abs(np.sin(t))
            return min(a / c if c > 0 else np.inf, b / s if s > 0 else np.inf)
        corner = np.arctan2(b, a)
        val = 4 * (quad(edge, 0, corner, epsabs=0, epsrel=1e-13)[0]
                   + quad(edge, corner, np.pi / 2, epsabs=0, epsrel=1e-13)[0])
        assert abs(W._rect_self_integral(a, b) - val) <= 1e-11 * val, (a, b)
