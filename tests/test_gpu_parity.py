"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Tolerances:
* tree keys and permutations: bit-exact;
* densities and Sommerfeld tables (FP64, plan time): 1e-12 relative to the largest
  value of the same degree N;
* the FP64 FMM: relative L2 error vs the direct-sum oracle, <= 1e-7 at p = 12 (the
  stated target), and the spectral decay with p at smaller orders.
"""
import math
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

D3 = [0.0, -1.0]
E3 = [1.0, 5.0, 2.0]


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def F():
    from paper_1908_10863_amd import fmmlm
    fmmlm.lib()
    return fmmlm


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def relerr(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


# ---------------------------------------------------------------- densities
@pytest.mark.parametrize("d,eps", [(D3, E3), ([0.0, -0.6, -1.4], [1.0, 3.9, 11.7, 2.5]),
                                   ([0.3], [2.0, 7.0]),
                                   ([0.0, -0.5, -1.0, -1.8, -2.6], [3.0, 1.5, 8.0, 11.0, 2.2, 6.5])])
def test_density_real_k(dev, F, oracle_mod, d, eps):
    _say(f"density real k L={len(d)}")
    L = len(d)
    ks = np.array([0.0, 0.01, 0.3, 1.0, 2.7, 9.0, 40.0])
    for lt in range(L + 1):
        for ls in range(L + 1):
            for a in (1, 2):
                for b in (1, 2):
                    if not (oracle_mod.valid(L, lt, a) and oracle_mod.valid(L, ls, b)):
                        continue
                    g = F.density(d, eps, lt, ls, a, b, ks)
                    o = np.array([oracle_mod.sigma(d, eps, lt, ls, k)[2 * (a - 1) + (b - 1)] for k in ks])
                    np.testing.assert_allclose(g.real, o, rtol=1e-13, atol=1e-14)
                    assert np.all(np.abs(g.imag) < 1e-15)


def test_density_imaginary_axis(dev, F, oracle_mod):
    """sigma(i eta) on the contour of eq. contourchange vs the mpmath interface solve."""
    _say("density imaginary axis")
    d, eps = [0.0, -0.6, -1.4], [1.0, 3.9, 11.7, 2.5]
    etas = [0.3, 2.0, 7.5]
    for (lt, ls, a, b) in [(0, 0, 1, 1), (1, 2, 2, 1), (3, 1, 2, 2), (2, 2, 1, 2)]:
        g = F.density(d, eps, lt, ls, a, b, 1j * np.array(etas))
        for e, v in zip(etas, g):
            ref = complex(oracle_mod.sigma_mp(d, eps, lt, ls, 1j * e, dps=25)[2 * (a - 1) + (b - 1)])
            assert abs(v - ref) < 1e-13 * max(1.0, abs(ref))


# ---------------------------------------------------------------- Sommerfeld tables
def _table31():
    rows = []
    with open(os.path.join(os.path.dirname(__file__), "golden", "table_3_1.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            rho, n, m, pts, err = line.split()
            rows.append((float(rho), int(n), int(m), int(pts), float(err)))
    return rows


def test_sommerfeld_table_3_1(dev, F, oracle_mod):
    """sigma == 1, z = 0.001, S = r (Table 3.1): the GPU quadrature (real axis for rho <= z,
    K_m contour otherwise) against the closed form, to the accuracy the paper prints for
    its DE-SE rule."""
    _say("sommerfeld table 3.1")
    for rho, n, m, _, err in _table31():
        z = 0.001
        S = math.hypot(rho, z)
        # initial values only (M = 0, 1) are quadratures; take the table at nmax = n
        tab = F.sommerfeld([], [], 0, 0, 1, 1, S, [rho], [z], n)[0]
        got = tab[n * (n + 1) // 2 + m]
        ref = oracle_mod.sommerfeld_sigma1(n, m, rho, z, S)
        assert abs(got - ref) <= max(10 * abs(err), 1e-12 * max(1.0, abs(ref))), (rho, n, m, got, ref)


@pytest.mark.parametrize("nmax", [16, 20, 24])
def test_sommerfeld_three_layer_tables(dev, F, oracle_mod, nmax):
    """Full S^N I_{N,M} tables at M2L geometries (rho in {0} U [S, sqrt(18) S], z in
    {1, 2, 3} S) for all 16 components against the image-series closed form.

    The forward recurrence carries an absolute error of order eps times the table's
    scale into every entry; when the density decays much faster than rho (large
    zeta_inf) the high orders are themselves far below that scale.  Since scaled
    multipole coefficients are O(1), that absolute error is what reaches the local
    expansion, so each row is judged by 3e-11 of its own largest entry plus 1e-14 of
    the whole table's largest entry."""
    _say(f"sommerfeld 3-layer nmax={nmax}")
    S = 0.1375
    geo = [(0.0, 1), (1.0, 1), (math.sqrt(2), 2), (math.sqrt(8), 1), (math.sqrt(18), 1), (3.0, 3)]
    rho = np.array([g[0] * S for g in geo])
    z = np.array([g[1] * S for g in geo])
    comps = [(lt, ls, a, b) for lt in range(3) for ls in range(3) for a in (1, 2) for b in (1, 2)
             if oracle_mod.valid(2, lt, a) and oracle_mod.valid(2, ls, b)]
    for (lt, ls, a, b) in comps:
        tab = F.sommerfeld(D3, E3, lt, ls, a, b, S, rho, z, nmax)
        for g in range(len(geo)):
            refs = [np.array([oracle_mod.sommerfeld_image3(D3, E3, lt, ls, a, b, N, M, rho[g], z[g], S)
                              for M in range(N + 1)]) for N in range(nmax + 1)]
            tmax = max(np.abs(r).max() for r in refs)
            for N in range(nmax + 1):
                got = tab[g, N * (N + 1) // 2: N * (N + 1) // 2 + N + 1]
                tol = 3e-11 * np.abs(refs[N]).max() + 1e-14 * tmax
                assert np.abs(got - refs[N]).max() <= tol, (lt, ls, a, b, g, N)


# ---------------------------------------------------------------- tree
@pytest.mark.parametrize("cfg,n", [(0, None), (1, 20000), (2, None)])
def test_tree_keys_bit_exact(dev, F, oracle_mod, cfg, n):
    from paper_1908_10863_amd import workloads as W
    # the last case is the benchmark's N = 1,048,576 (hundreds of radix-sort tiles per tree)
    _say(f"tree keys cfg={cfg}")
    w = W.config(cfg, n=n)
    plan = F.Plan(w["d"], w["eps"], w["x"], w["y"], w["z"], w["layer"], p=4, leaf_cap=w["leaf_cap"])
    st = plan.stats()
    scale = np.ldexp(1.0, 21) / st["root_side"]
    d = w["d"]
    for t in range(st["n_trees"]):
        layer, side, keys, perm = plan.tree(t)
        members = np.nonzero(w["layer"] == layer)[0]
        h = (w["z"][members] - d[layer]) if side == 1 else (d[layer - 1] - w["z"][members])
        ok = oracle_mod.morton_keys(w["x"][members], w["y"][members], h, st["x0"], st["y0"], scale)
        sk, sp = oracle_mod.morton_sort(ok)
        assert np.array_equal(keys, sk)
        assert np.array_equal(perm, members[sp])
    plan.close()


# ---------------------------------------------------------------- FMM end to end
def _run(F, w, p, dev, parts=3, leaf_cap=None, q=None):
    import torch
    plan = F.Plan(w["d"], w["eps"], w["x"], w["y"], w["z"], w["layer"], p=p,
                  leaf_cap=leaf_cap or w["leaf_cap"])
    qq = torch.tensor(w["q"][0] if q is None else q, dtype=torch.float64, device=dev)
    phi = plan.eval(qq, parts=parts).cpu().numpy()
    st = plan.stats()
    plan.close()
    return phi, st


def test_config1_p8_full_oracle(dev, F, oracle_mod):
    """Workload 1 (N = 1200, p = 8, <= 40 per leaf) against the full N^2 direct sum,
    free and reaction parts separately and together."""
    from paper_1908_10863_amd import workloads as W
    _say("config1 p=8")
    w = W.config(0)
    args = (w["d"], w["eps"], w["x"], w["y"], w["z"], w["layer"], w["q"][0])
    ref_f = oracle_mod.potential(*args, parts=1)
    ref_r = oracle_mod.potential(*args, parts=2)
    phi_f, st = _run(F, w, 8, dev, parts=1)
    phi_r, _ = _run(F, w, 8, dev, parts=2)
    phi, _ = _run(F, w, 8, dev, parts=3)
    ef, er, et = relerr(phi_f, ref_f), relerr(phi_r, ref_r), relerr(phi, ref_f + ref_r)
    nf, nr = np.linalg.norm(ref_f), np.linalg.norm(ref_r)
    _say(f"  free {ef:.3e} reaction {er:.3e} total {et:.3e} (absolute {ef * nf:.3e}, {er * nr:.3e}) stats {st}")
    # Truncation at p = 8, MAC 6 (measured 1.63e-6 free, 1.81e-6 total).  Both parts pass
    # through the same expansions at the same p and MAC, so their absolute errors are
    # alike; the reaction part is held to the free part's bound in absolute terms
    # (its norm is 1/4.86 of the free part's, so its relative error is ~5x larger).
    assert ef < 5e-6 and et < 5e-6
    assert er * nr < 5e-6 * nf
    np.testing.assert_allclose(phi_f + phi_r, phi, rtol=0, atol=1e-12 * np.abs(phi).max())


def test_config1_p12_meets_1e7(dev, F, oracle_mod):
    from paper_1908_10863_amd import workloads as W
    _say("config1 p=12")
    w = W.config(0)
    ref = oracle_mod.potential(w["d"], w["eps"], w["x"], w["y"], w["z"], w["layer"], w["q"][0])
    phi, _ = _run(F, w, 12, dev)
    e = relerr(phi, ref)
    _say(f"  p=12 rel L2 {e:.3e}")
    assert e <= 1e-7


def test_spectral_convergence_in_p(dev, F, oracle_mod):
    """Errors fall geometrically with p (Sec. 4, Fig. fmmconvergence (b) analogue)."""
    from paper_1908_10863_amd import workloads as W
    _say("convergence in p")
    w = W.config(0)
    ref = oracle_mod.potential(w["d"], w["eps"], w["x"], w["y"], w["z"], w["layer"], w["q"][0])
    errs = []
    for p in (2, 4, 6, 8, 10):
        phi, _ = _run(F, w, p, dev)
        errs.append(relerr(phi, ref))
    _say(f"  errors {errs}")
    for a, b in zip(errs, errs[1:]):
        assert b < 0.5 * a
    assert errs[-1] < 1e-6


def test_every_order(dev, F, oracle_mod):
    """Every truncation order p = 1..16 (the kernels with the order fixed at compile time,
    P2M and L2P, have one instantiation each, and the M2L tiles one row count per few
    orders): the FP64 form's error does not grow from one order to the next and is
    below 1e-8 at p = 16; the FP32 form stays within its rounding floor of the FP64 form."""
    import torch
    from paper_1908_10863_amd import workloads as W
    _say("every order p = 1..16")
    w = W.config(0)
    ref = oracle_mod.potential(w["d"], w["eps"], w["x"], w["y"], w["z"], w["layer"], w["q"][0])
    q = torch.tensor(w["q"][0], dtype=torch.float64, device=dev)
    e64, e32 = [], []
    for p in range(1, 17):
        for prec, out in ((F.FMMLM_FP64, e64), (F.FMMLM_FP32_COMPENSATED, e32)):
            plan = F.Plan(w["d"], w["eps"], w["x"], w["y"], w["z"], w["layer"], p=p,
                          leaf_cap=w["leaf_cap"], precision=prec)
            out.append(relerr(plan.eval(q).cpu().numpy(), ref))
            plan.close()
        _say(f"  p={p:2d} fp64 {e64[-1]:.2e} fp32 {e32[-1]:.2e}")
    for p in range(2, 17):
        assert e64[p - 1] <= 1.5 * e64[p - 2] + 1e-12, p
    assert e64[-1] < 1e-8
    for a, b in zip(e64, e32):
        assert b <= a + 3e-6


def test_largest_order_p16(dev, F, oracle_mod):
    """The largest truncation order (p = 16, FP64 form, default MAC) against the full
    direct sum: more accurate than p = 12's 1e-7 bound."""
    from paper_1908_10863_amd import workloads as W
    _say("p = 16")
    w = W.config(0)
    ref = oracle_mod.potential(w["d"], w["eps"], w["x"], w["y"], w["z"], w["layer"], w["q"][0])
    phi, st = _run(F, w, 16, dev)
    e = relerr(phi, ref)
    _say(f"  rel L2 {e:.2e}, {st['m2l_free_pairs']} + {st['m2l_reaction_pairs']} M2L pairs")
    assert st["m2l_free_pairs"] > 0 and st["m2l_reaction_pairs"] > 0
    assert e < 1e-7


def test_largest_stack_twelve_interfaces(dev, F, oracle_mod):
    """The largest medium (12 interfaces, 13 layers, seeded permittivities in [1, 12]):
    FP64 form p = 10 with 8 points a leaf (expansions carry most pairs) against the
    quadrature direct sum on 130 targets."""
    from paper_1908_10863_amd import workloads as W
    _say("12 interfaces")
    d = [-0.3 * i for i in range(12)]
    eps = list(np.random.default_rng(31).uniform(1.0, 12.0, 13))
    w = W.make_layered(d, eps, W.split_even(390, 13), 32)
    w["leaf_cap"] = 8
    t = np.arange(0, 390, 3)
    ref = oracle_mod.potential(d, eps, w["x"], w["y"], w["z"], w["layer"], w["q"][0], targets=t, method="quad")
    phi, st = _run(F, w, 10, dev)
    e = relerr(phi[t], ref)
    _say(f"  rel L2 {e:.2e}, {st['n_trees']} trees, {st['m2l_reaction_pairs']} reaction M2L pairs")
    assert st["n_trees"] == 24 and st["m2l_reaction_pairs"] > 0
    assert e < 1e-6


def test_contour_form_resolves_the_whole_stack(dev, F, oracle_mod):
    """Regression: along the imaginary axis a density keeps the oscillation of a
    round trip through the whole stack; with 12 thin layers the contour form's
    panels must resolve it (same-layer component at rho > zeta, where the
    contour form applies), against the oracle's real-axis quadrature."""
    d = [-0.3 * i for i in range(12)]
    eps = list(np.random.default_rng(31).uniform(1.0, 12.0, 13))
    for (a, b, zeta) in [(1, 1, 0.225), (2, 2, 0.375), (1, 2, 0.307)]:
        for rho in (0.5, 0.838, 1.3):
            g = F.sommerfeld(d, eps, 6, 6, a, b, 1.0, [rho], [zeta], 0)[0, 0]
            o = oracle_mod.reaction_quad(d, eps, 6, 6, a, b, rho, zeta) * 4 * math.pi
            assert abs(g - o) <= 1e-7 * abs(o), (a, b, zeta, rho, g, o)


def test_points_hugging_an_interface(dev, F, oracle_mod):
    """Two thirds of the points within 1e-4..2e-3 of the top interface, on both
    sides (tiny zeta for the reaction self and near terms), three layers: FP64 p = 12
    <= 1e-7 and the FP32 form <= 1e-5 against the image-series direct sum."""
    import torch
    d, eps = D3, E3
    rng = np.random.default_rng(61)
    n = 3000
    lay = np.repeat([0, 1, 2], n // 3).astype(np.int32)
    z = np.where(lay == 0, rng.uniform(1e-4, 2e-3, n),
                 np.where(lay == 1, rng.uniform(-2e-3, -1e-4, n), rng.uniform(-1.5, -1.1, n)))
    x, y, q = rng.uniform(-0.5, 0.5, n), rng.uniform(-0.5, 0.5, n), rng.uniform(-1, 1, n)
    ref = oracle_mod.potential(d, eps, x, y, z, lay, q, method="image3")
    for prec, p, mac, tol in [(0, 12, 6, 1e-7), (1, 10, 4, 1e-5)]:
        pl = F.Plan(d, eps, x, y, z, lay, p=p, leaf_cap=40, precision=prec, mac_d2=mac)
        phi = pl.eval(torch.tensor(q, device=dev)).cpu().numpy()
        pl.close()
        e = relerr(phi, ref)
        _say(f"  hugging the interface, precision {prec}: {e:.2e}")
        assert e < tol


def test_scale_and_translation_invariance(dev, F):
    """Lengths scaled by s give potentials scaled by 1/s, and a lateral shift
    changes nothing (no absolute length hides in the plan: an inverse-length
    panel bound once written as a length made a 1e-3 scale take effectively
    forever).  FP64 form p = 12 and the FP32 form."""
    import torch
    from paper_1908_10863_amd import workloads as W
    w = W.config(0, n=3000, seed=71)
    q = torch.tensor(w["q"][0], device=dev)

    def run(d, x, y, z, prec):
        kw = dict(p=12, leaf_cap=40, mac_d2=6) if prec == 0 else dict(p=10, leaf_cap=40, mac_d2=4, precision=1)
        pl = F.Plan(d, w["eps"], x, y, z, w["layer"], **kw)
        phi = pl.eval(q).cpu().numpy()
        pl.close()
        return phi

    for prec, tol_s, tol_t in [(0, 1e-12, 1e-9), (1, 1e-6, 1e-7)]:
        base = run(w["d"], w["x"], w["y"], w["z"], prec)
        for s in (1e-3, 1e3):
            _say(f"  precision {prec}, lengths x {s:g}")
            phi = run([v * s for v in w["d"]], w["x"] * s, w["y"] * s, w["z"] * s, prec) * s
            assert relerr(phi, base) < tol_s, (prec, s)
        phi = run(w["d"], w["x"] + 1e4, w["y"] - 1e4, w["z"], prec)
        assert relerr(phi, base) < tol_t, prec


def test_charges_on_one_vertical_line(dev, F, oracle_mod):
    """Every pair at rho = 0 (all points at x = y = 0, random heights in three
    layers): the rho = 0 paths of the Sommerfeld integrals (orders m > 0 vanish),
    M2L offsets on the axis and a deep tree.  FP64 form p = 12, default MAC,
    against the image-series direct sum."""
    import torch
    rng = np.random.default_rng(81)
    n = 1500
    lay = np.repeat([0, 1, 2], n // 3).astype(np.int32)
    zr = {0: (0.1, 1.1), 1: (-0.9, -0.1), 2: (-2.0, -1.1)}
    z = np.array([rng.uniform(*zr[int(v)]) for v in lay])
    x = np.zeros(n)
    q = rng.uniform(-1, 1, n)
    ref = oracle_mod.potential(D3, E3, x, x, z, lay, q, method="image3")
    pl = F.Plan(D3, E3, x, x, z, lay, p=12, leaf_cap=20)
    phi = pl.eval(torch.tensor(q, device=dev)).cpu().numpy()
    st = pl.stats()
    pl.close()
    e = relerr(phi, ref)
    _say(f"  vertical line: {e:.2e}, {st['max_level']} levels")
    assert st["max_level"] >= 6
    assert e < 1e-9


def test_charges_on_one_vertical_line_fp32(dev, F, oracle_mod):
    """The same input in the FP32 form at the benchmark's settings (p = 10, mac_d2 = 4): a
    documented limit of that form.  The closest pairs are about 4e-6 apart, below the
    resolution of a leaf-relative FP32 coordinate difference on these deep leaves, and
    mac_d2 = 4 leaves a worst-case reaction truncation near 1e-4 for boxes on one axis;
    the test records the error and holds it to the level measured when the limit was
    documented (1.6e-4), not to the form's 1e-5 for uniform boxes."""
    import torch
    rng = np.random.default_rng(81)
    n = 1500
    lay = np.repeat([0, 1, 2], n // 3).astype(np.int32)
    zr = {0: (0.1, 1.1), 1: (-0.9, -0.1), 2: (-2.0, -1.1)}
    z = np.array([rng.uniform(*zr[int(v)]) for v in lay])
    x = np.zeros(n)
    q = rng.uniform(-1, 1, n)
    out = {}
    for parts in (1, 2, 3):
        ref = oracle_mod.potential(D3, E3, x, x, z, lay, q, method="image3", parts=parts)
        pl = F.Plan(D3, E3, x, x, z, lay, p=10, leaf_cap=20, precision=F.FMMLM_FP32_COMPENSATED, mac_d2=4)
        phi = pl.eval(torch.tensor(q, device=dev), parts=parts).cpu().numpy()
        pl.close()
        out[parts] = relerr(phi, ref)
    _say(f"  vertical line, FP32 form p=10 mac 4: free {out[1]:.2e} reaction {out[2]:.2e} total {out[3]:.2e}")
    assert out[3] < 3e-4
    assert out[1] < 3e-4 and out[2] < 3e-4


def test_high_contrast_medium(dev, F, oracle_mod):
    """eps = (1, 80, 1): reflections of magnitude 0.975 give the density sharp
    resonances along the imaginary axis.  The contour form's integrals stay within
    2e-5 of the oracle's real-axis quadrature (a known limit of its panels), and the
    FMM still meets 1e-7 at p = 12 against the image-series direct sum."""
    import torch
    from paper_1908_10863_amd import workloads as W
    d, eps = [0.0, -1.0], [1.0, 80.0, 1.0]
    worst = 0.0
    for c in [(0, 0, 1, 1), (1, 1, 1, 2), (1, 2, 1, 2), (2, 1, 2, 1), (1, 1, 2, 2)]:
        zinf = F.density_asymptotic(d, eps, *c)[1]
        for zeta in (0.05, 0.5):
            for rho in (0.8, 3.0):
                if rho <= zeta + zinf:
                    continue
                g = F.sommerfeld(d, eps, *c, 1.0, [rho], [zeta], 0)[0, 0]
                o = oracle_mod.reaction_quad(d, eps, c[0], c[1], c[2], c[3], rho, zeta) * 4 * math.pi
                worst = max(worst, abs(g - o) / abs(o))
    _say(f"  high contrast: worst contour-form integral {worst:.1e}")
    assert worst < 2e-5
    w = W.make_layered(d, eps, W.split_even(1200, 3), 41)
    ref = oracle_mod.potential(d, eps, w["x"], w["y"], w["z"], w["layer"], w["q"][0], method="image3")
    pl = F.Plan(d, eps, w["x"], w["y"], w["z"], w["layer"], p=12, leaf_cap=40)
    phi = pl.eval(torch.tensor(w["q"][0], device=dev)).cpu().numpy()
    pl.close()
    assert relerr(phi, ref) < 1e-7


def test_four_layer_quadrature_oracle(dev, F, oracle_mod):
    """A four-layer medium (workload 4's interfaces) at small N against the quadrature
    oracle (no closed form used anywhere)."""
    from paper_1908_10863_amd import workloads as W
    _say("four layers")
    w = W.config(3, n=600)
    t = np.arange(0, 600, 5)
    ref = oracle_mod.potential(w["d"], w["eps"], w["x"], w["y"], w["z"], w["layer"], w["q"][0],
                               targets=t, method="quad")
    phi, st = _run(F, w, 12, dev, leaf_cap=20)
    e = relerr(phi[t], ref)
    _say(f"  rel L2 {e:.3e} m2l_reaction {st['m2l_reaction_pairs']}")
    assert e < 1e-7


def test_two_layer_close_to_interface(dev, F, oracle_mod):
    """Points close to a single interface exercise the reaction near field (P2P with
    per-pair Sommerfeld kernels)."""
    _say("two layers near interface")
    rng = np.random.default_rng(9)
    n = 800
    lay = (rng.uniform(size=n) < 0.5).astype(np.int32)
    x = rng.uniform(-0.5, 0.5, n)
    y = rng.uniform(-0.5, 0.5, n)
    z = np.where(lay == 0, rng.uniform(0.002, 0.3, n), -rng.uniform(0.002, 0.3, n))
    w = dict(d=np.array([0.0]), eps=np.array([2.0, 9.0]), x=x, y=y, z=z, layer=lay,
             q=rng.uniform(-1, 1, (1, n)), leaf_cap=16)
    t = np.arange(0, n, 4)
    ref = oracle_mod.potential(w["d"], w["eps"], x, y, z, lay, w["q"][0], targets=t, method="quad")
    phi, st = _run(F, w, 12, dev)
    _say(f"  reaction near pairs {st['p2p_reaction_pairs']}")
    assert st["p2p_reaction_pairs"] > 0
    assert relerr(phi[t], ref) < 1e-7


@pytest.mark.parametrize("d,eps", [([0.0], [2.0, 9.0]), (D3, E3), ([0.0, -0.6, -1.4], [1.0, 3.9, 11.7, 2.5])])
def test_near_field_kernel_values(dev, F, oracle_mod, d, eps):
    """I_00 / 4pi at near-field geometries (small rho and zeta, both quadrature paths)
    against the oracle's kernel: the values the plan stores for reaction P2P."""
    _say(f"near-field kernels L={len(d)}")
    L = len(d)
    rhos = np.array([0.0, 0.001, 0.01, 0.05, 0.3])
    for zeta in (0.004, 0.01, 0.1, 0.5):
        for lt in range(L + 1):
            for ls in range(L + 1):
                for a in (1, 2):
                    for b in (1, 2):
                        if not (oracle_mod.valid(L, lt, a) and oracle_mod.valid(L, ls, b)):
                            continue
                        got = F.sommerfeld(d, eps, lt, ls, a, b, 1.0, rhos, np.full(len(rhos), zeta), 0)[:, 0]
                        ref = np.array([4 * math.pi * oracle_mod.reaction_quad(d, eps, lt, ls, a, b, r, zeta)
                                        for r in rhos])
                        # GPU graded rule and oracle fixed rule agree to 2.4e-15 here (four layers)
                        np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-14 * np.abs(ref).max())


def test_pure_near_field_matches_direct_sum(dev, F, oracle_mod):
    """With one leaf per tree nothing goes through expansions: the free part is the P2P
    kernel alone and the reaction part the stored near-field kernels alone."""
    from paper_1908_10863_amd import workloads as W
    _say("pure near field")
    w = W.config(0, n=450)
    args = (w["d"], w["eps"], w["x"], w["y"], w["z"], w["layer"], w["q"][0])
    for parts in (1, 2):
        phi, st = _run(F, w, 4, dev, parts=parts, leaf_cap=1000)
        assert st["m2l_free_pairs"] == 0 and st["m2l_reaction_pairs"] == 0
        ref = oracle_mod.potential(*args, parts=parts)
        assert relerr(phi, ref) < 1e-13


@pytest.mark.parametrize("precision,n,cap", [(0, 2400, 220), (1, 2400, 220), (0, 6400, 500), (1, 6400, 500)])
def test_near_field_pairs_both_ways(dev, F, oracle_mod, precision, n, cap):
    """One interface, each layer's points filling its tree's root cube: the free-space
    trees stop at depth one, the eight leaves of a tree are mutually adjacent, and every
    free-space pair is near field.  A pair of distinct leaves is evaluated once for both
    of its sums; leaves of about n/16 points span several work units (128 targets in
    the FP32 form, 64 in FP64).  The free part equals the direct sum."""
    import torch
    _say(f"near field both ways precision={precision} n={n} cap={cap}")
    rng = np.random.default_rng(31 + n)
    h = n // 2
    x = rng.uniform(-0.5, 0.5, n)
    y = rng.uniform(-0.5, 0.5, n)
    z = np.concatenate([rng.uniform(1e-3, 1.0, h), -rng.uniform(1e-3, 1.0, n - h)])
    layer = np.concatenate([np.zeros(h, np.int32), np.ones(n - h, np.int32)])
    d, eps = np.array([0.0]), np.array([1.0, 3.0])
    qv = rng.uniform(-1, 1, n)
    plan = F.Plan(d, eps, x, y, z, layer, p=8, leaf_cap=cap, precision=precision)
    st = plan.stats()
    phi = plan.eval(torch.tensor(qv, dtype=torch.float64, device=dev), parts=1).cpu().numpy()
    plan.close()
    assert st["m2l_free_pairs"] == 0
    assert st["p2p_free_pairs"] == h * h + (n - h) * (n - h)  # every ordered pair, self pairs included
    ref = oracle_mod.potential(d, eps, x, y, z, layer, qv, parts=1)
    e = relerr(phi, ref)
    _say(f"  {e:.3e}")
    assert e < (1e-13 if precision == 0 else 2e-6)


def test_homogeneous_medium_is_coulomb(dev, F):
    """All permittivities equal: the layered FMM reproduces the plain Coulomb sum over
    all charges across layers."""
    from paper_1908_10863_amd import workloads as W
    _say("homogeneous")
    w = W.config(0, n=900)
    w["eps"] = np.array([3.0, 3.0, 3.0])
    P = np.stack([w["x"], w["y"], w["z"]], 1)
    R = np.linalg.norm(P[:, None] - P[None], axis=2)
    np.fill_diagonal(R, np.inf)
    ref = (w["q"][0][None, :] / (4 * math.pi * R)).sum(1)
    phi, _ = _run(F, w, 12, dev)
    assert relerr(phi, ref) < 1e-7


def test_multiple_rhs_and_determinism(dev, F):
    import torch
    from paper_1908_10863_amd import workloads as W
    _say("multi rhs")
    w = W.config(0, n=600)
    plan = F.Plan(w["d"], w["eps"], w["x"], w["y"], w["z"], w["layer"], p=6, leaf_cap=30, max_rhs=3)
    plan.set_variants(batch_min=2)  # the batched pass, whatever the tuner measured
    rng = np.random.default_rng(1)
    Q = torch.tensor(rng.uniform(-1, 1, (3, 600)), dtype=torch.float64, device=dev)
    both = plan.eval(Q).cpu().numpy()
    for r in range(3):
        one = plan.eval(Q[r].contiguous()).cpu().numpy()
        # batched and single-vector passes sum in different orders
        np.testing.assert_allclose(both[r], one, rtol=0, atol=1e-13 * np.abs(one).max())
    again = plan.eval(Q).cpu().numpy()
    assert np.array_equal(again, both)
    # linearity
    lin = plan.eval((2.0 * Q[0] - Q[1]).contiguous()).cpu().numpy()
    np.testing.assert_allclose(lin, 2 * both[0] - both[1], rtol=0, atol=1e-12 * np.abs(lin).max())
    plan.close()


def test_tiny_and_ragged_inputs(dev, F, oracle_mod):
    """One charge, two charges, an empty layer, and a leaf cap of 1 (every pair that can
    go through expansions does)."""
    import torch
    _say("tiny inputs")
    cases = [
        (np.array([0.1]), np.array([0.2]), np.array([0.5]), np.array([0]), 8),
        (np.array([0.1, -0.2]), np.array([0.2, 0.0]), np.array([0.5, -0.4]), np.array([0, 1]), 1),
        (np.array([0.1, -0.2, 0.3]), np.array([0.2, 0.0, -0.1]), np.array([0.5, 0.6, -1.5]),
         np.array([0, 0, 2]), 1),
    ]
    for x, y, z, lay, cap in cases:
        q = np.linspace(-1, 1, len(x)) + 0.3
        ref = oracle_mod.potential(D3, E3, x, y, z, lay, q)
        err = {}
        for p in (8, 12):
            plan = F.Plan(D3, E3, x, y, z, lay, p=p, leaf_cap=cap)
            phi = plan.eval(torch.tensor(q, dtype=torch.float64, device=dev)).cpu().numpy()
            st = plan.stats()
            plan.close()
            err[p] = np.abs(phi - ref) / np.abs(ref)
            far = st["m2l_free_pairs"] + st["m2l_reaction_pairs"]
        _say(f"  n={len(x)} cap={cap} M2L pairs {far}: p=8 {err[8]}, p=12 {err[12]}")
        if far == 0:
            # pure near field: nothing is truncated, only rounding remains
            assert err[8].max() < 1e-13 and err[12].max() < 1e-13
        else:
            # element by element: truncation at p = 8 (measured 6.8e-8 on the one reaction
            # M2L pair) and, from p = 8 to 12, at least the geometric decay (1/sqrt(2))^4 of
            # eq. meerror's rate for boxes separated by mac_d2 = 6 ((a_s + a_t) / R <=
            # sqrt(3) / sqrt(6)); points in leaves of their own keep rounding
            assert err[8].max() < 1e-6
            assert np.all(err[12] <= err[8] * 0.5 ** 2 + 1e-13)


@pytest.mark.parametrize("cfg,p,tol", [(1, 12, 1e-7), (2, 10, 1e-6)])
def test_full_size_sampled(dev, F, oracle_mod, cfg, p, tol):
    """Workloads 2 (N = 262144, clustered middle layer) and 3 (N = 1048576) at full size,
    checked on 64 sampled targets against the direct sum over all N sources."""
    from paper_1908_10863_amd import workloads as W
    _say(f"full size cfg={cfg} p={p}")
    w = W.config(cfg)
    rng = np.random.default_rng(123)
    t = np.sort(rng.choice(len(w["x"]), 64, replace=False))
    ref = oracle_mod.potential(w["d"], w["eps"], w["x"], w["y"], w["z"], w["layer"], w["q"][0],
                               targets=t)
    phi, st = _run(F, w, p, dev)
    e = relerr(phi[t], ref)
    _say(f"  rel L2 {e:.3e} plan {st['plan_seconds']:.2f}s boxes {st['n_boxes']}")
    assert e <= tol
