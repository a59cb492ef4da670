"""Pins of the oracle's densities and direct sum for the general interface
conditions of App. A (a u and b du/dz continuous at every interface).

* a = 1, b = eps gives the classic densities bit for bit.
* Half-space closed forms (one interface, any k): reflection
  (b0 a1 - b1 a0) / (b0 a1 + b1 a0) and transmission 2 a0 b0 / (b0 a1 + b1 a0),
  from matching the free wave and its image across the interface.
* Only ratios matter: scaling every a (or every b) by one constant leaves the
  densities unchanged.
* The weighted reciprocity of the general problem, a_i b_i G_ij symmetric
  (for a = 1 it is the classic eps_i G_ij), on the direct sum.
"""
import numpy as np
import pytest

import oracle

D4 = [0.0, -0.6, -1.4]


def test_classic_is_the_special_case():
    eps = [1.0, 3.9, 11.7, 2.5]
    for lt in range(4):
        for ls in range(4):
            for k in (0.05, 1.3, 7.0):
                assert np.array_equal(oracle.sigma_ab(D4, [1.0] * 4, eps, lt, ls, k),
                                      oracle.sigma(D4, eps, lt, ls, k))


@pytest.mark.parametrize("a,b", [((1.0, 1.0), (1.0, 4.0)), ((1.7, 0.6), (2.0, 0.9)), ((0.3, 2.2), (5.0, 5.0))])
def test_half_space_closed_form(a, b):
    a0, a1 = a
    b0, b1 = b
    R = (b0 * a1 - b1 * a0) / (b0 * a1 + b1 * a0)
    T = 2 * a0 * b0 / (b0 * a1 + b1 * a0)
    for k in (0.1, 2.0, 9.0):
        refl = oracle.sigma_ab([0.0], a, b, 0, 0, k)   # source and target above
        tran = oracle.sigma_ab([0.0], a, b, 1, 0, k)   # target below
        # one nonzero entry each: the image above, the transmitted wave below
        assert np.count_nonzero(refl) == 1 and np.count_nonzero(tran) == 1
        assert abs(refl[refl != 0][0] - R) <= 1e-14
        assert abs(tran[tran != 0][0] - T) <= 1e-14


def test_only_ratios_matter():
    rng = np.random.default_rng(3)
    a = rng.uniform(0.3, 3.0, 4)
    b = rng.uniform(0.5, 8.0, 4)
    for lt in range(4):
        for ls in range(4):
            k = float(rng.uniform(0.05, 5.0))
            s = oracle.sigma_ab(D4, a, b, lt, ls, k)
            s2 = oracle.sigma_ab(D4, 2.5 * a, 0.4 * b, lt, ls, k)
            assert np.abs(s - s2).max() <= 1e-13 * max(1.0, np.abs(s).max())


def test_weighted_reciprocity_of_the_direct_sum():
    rng = np.random.default_rng(4)
    a = np.array([1.0, 0.5, 2.0, 1.5])
    b = np.array([1.0, 3.0, 6.0, 1.2])
    n = 10
    lay = np.array([0, 1, 2, 3, 1, 2, 0, 3, 2, 1], np.int32)
    lo = np.array([0.1, -0.5, -1.3, -2.4])
    hi = np.array([1.0, -0.1, -0.7, -1.5])
    z = rng.uniform(lo[lay], hi[lay])
    x = rng.uniform(-0.5, 0.5, n)
    y = rng.uniform(-0.5, 0.5, n)
    G = np.zeros((n, n))
    for j in range(n):
        q = np.zeros(n)
        q[j] = 1.0
        G[:, j] = oracle.potential_ab(D4, a, b, x, y, z, lay, q, parts=2)
    W = (a * b)[lay][:, None] * G
    assert np.abs(W - W.T).max() <= 1e-10 * np.abs(W).max()
    # the unweighted operator is not symmetric
    assert np.abs(G - G.T).max() > 1e-3 * np.abs(G).max()
