"""Table form of the Sommerfeld initial values (the Remark after Table 3.1).

* The interpolation kernel on host-given node values: exact (to rounding) for
  polynomials of degree <= 11 in each variable on every panel, and not exact at
  degree 12 (so the stated degree is the kernel's).
* The tables of a medium against the quadrature, in interaction units
  R1 max_{N,M} 0.87^N |difference| (as for the learned form), at M2L geometry.
* The FMM with the tables against the direct-sum oracle, and against the FMM with
  the quadrature: the tables keep the FP64 form's accuracy (<= 1e-7 at p = 12).
* Plan time with the tables against the quadrature and the network.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

D3 = [0.0, -1.0]
E3 = [1.0, 5.0, 2.0]
K = 12


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def relerr(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _nodes():
    k = np.arange(K)
    return np.cos((2 * k + 1) * np.pi / (2 * K))


def _poly(c, r, z):
    # sum c[a, b] r^a z^b (Horner in both variables)
    out = np.zeros_like(r)
    for a in range(c.shape[0] - 1, -1, -1):
        row = np.zeros_like(z)
        for b in range(c.shape[1] - 1, -1, -1):
            row = row * z + c[a, b]
        out = out * r + row
    return out


def test_interp2d_exact_on_polynomials():
    """Degree 11 in each variable, a different polynomial on every panel and output: exact
    to rounding at points inside panels, on panel edges and at nodes.  Degree 12 on one
    panel: x^12 is off by T_12(x) / 2^11 (the first-kind node polynomial), so the stated
    degree is the kernel's."""
    from paper_1908_10863_amd import fmmlm
    npr, npz, rmax, zmax, nout, deg = 3, 2, 1.3, 0.9, 3, 11
    hr, hz = rmax / npr, zmax / npz
    rng = np.random.default_rng(5)
    coef = rng.normal(0, 1, (npr, npz, nout, deg + 1, deg + 1))
    xk = _nodes()
    nodes = np.zeros((npr * npz, nout, K * K))
    for i in range(npr):
        for j in range(npz):
            r = (i + 0.5 + 0.5 * xk) * hr
            z = (j + 0.5 + 0.5 * xk) * hz
            R, Z = np.meshgrid(r, z, indexing="ij")
            for o in range(nout):
                nodes[i * npz + j, o] = _poly(coef[i, j, o], R, Z).ravel()
    n = 600
    rho = rng.uniform(0, rmax, n)
    zeta = rng.uniform(0, zmax, n)
    rho[:6] = [0.0, hr, 2 * hr, rmax, 0.5 * hr, (0.5 + 0.5 * xk[3]) * hr]   # edges and a node
    zeta[:6] = [0.0, hz, zmax, 0.3, (1.5 + 0.5 * xk[7]) * hz, (0.5 + 0.5 * xk[2]) * hz]
    got = fmmlm.interp2d(npr, npz, rmax, zmax, nodes, rho, zeta)
    pi = np.minimum((rho / hr).astype(int), npr - 1)
    pj = np.minimum((zeta / hz).astype(int), npz - 1)
    want = np.array([[_poly(coef[pi[m], pj[m], o], rho[m:m + 1], zeta[m:m + 1])[0] for o in range(nout)]
                     for m in range(n)])
    err = np.max(np.abs(got - want) / (1.0 + np.abs(want)))
    _say(f"  degree 11: max deviation {err:.2e}")
    assert err < 1e-12
    # degree 12 on [0, 2]^2: f = (r - 1)^12, local x = r - 1
    R, Z = np.meshgrid(1.0 + xk, 1.0 + xk, indexing="ij")
    nd = ((R - 1.0) ** 12).reshape(1, 1, K * K)
    x = np.linspace(-1, 1, 401)
    g = fmmlm.interp2d(1, 1, 2.0, 2.0, nd, 1.0 + x, np.full(len(x), 0.7))[:, 0]
    dev = x ** 12 - g
    np.testing.assert_allclose(dev, np.cos(12 * np.arccos(x)) / 2 ** 11, rtol=0, atol=1e-13)


def _m2l_geometry(rng, n, rmax, zmax):
    rho = rng.uniform(0, rmax, n)
    rho[: n // 8] = 0.0
    z = rng.uniform(0.02, zmax, n)
    S = 0.4 * np.hypot(rho, z)
    S = np.where(rho > 0, np.minimum(S, rho), S)
    return rho, z, S


def _interaction_error(got, ref, R1, nmax):
    nn = np.array([n for n in range(nmax + 1) for m in range(n + 1)])
    return float((np.abs(got - ref) * 0.87 ** nn * R1).max())


@pytest.mark.parametrize("medium", ["three", "six"])
def test_tables_against_quadrature(medium):
    from paper_1908_10863_amd import fmmlm, workloads as W
    if medium == "three":
        d, eps = D3, E3
        comps = [(1, 1, 1, 1), (0, 2, 1, 2), (2, 1, 2, 2), (1, 1, 2, 1)]
    else:
        w = W.config(4, n=64)
        d, eps = w["d"], w["eps"]
        comps = [(0, 0, 1, 1), (2, 3, 2, 1), (5, 1, 2, 2), (1, 4, 1, 2), (3, 3, 1, 2)]
    rmax, zmax = 1.6, 2.3
    tab = fmmlm.Surrogate(d, eps, p=10, rho_max=rmax, zeta_max=zmax, tables=True)
    info = tab.table_info()
    _say(f"  {medium}: tables {info}")
    rng = np.random.default_rng(3)
    rho, z, S = _m2l_geometry(rng, 120, rmax, zmax)
    worst = 0.0
    for (lt, ls, a, b) in comps:
        zi = fmmlm.density_asymptotic(d, eps, lt, ls, a, b)[1]
        for i in range(len(rho)):
            ref = fmmlm.sommerfeld(d, eps, lt, ls, a, b, S[i], rho[i:i + 1], z[i:i + 1], 20)
            got, used = tab.eval(lt, ls, a, b, S[i], rho[i:i + 1], z[i:i + 1], 20)
            assert used.all()
            worst = max(worst, _interaction_error(got, ref, np.hypot(rho[i], z[i] + zi), 20))
        # near-field kernel (N = 0) at small rho and zeta
        rr = np.array([0.0, 1e-3, 0.02, 0.1])
        zz = np.array([0.004, 0.03, 0.2, 0.6])
        for zv in zz:
            ref = fmmlm.sommerfeld(d, eps, lt, ls, a, b, 1.0, rr, np.full(4, zv), 0)[:, 0]
            got, used = tab.eval(lt, ls, a, b, 1.0, rr, np.full(4, zv), 0)
            worst = max(worst, float(np.max(np.abs(got[:, 0] - ref) * np.hypot(rr, zv + zi))))
    _say(f"  {medium}: worst interaction error {worst:.2e}")
    assert worst < 1e-10
    tab.close()


def test_fmm_with_tables_vs_oracle(oracle_mod):
    import torch
    from paper_1908_10863_amd import fmmlm, workloads as W
    q = None
    out = {}
    # six regions, FP64 form p = 10, against the quadrature direct sum
    w = W.config(4, n=1500, seed=77)
    t = np.arange(0, 1500, 25)
    ref = oracle_mod.potential(w["d"], w["eps"], w["x"], w["y"], w["z"], w["layer"], w["q"][0], targets=t,
                               method="quad")
    q = torch.tensor(w["q"][0], device="cuda:0")
    probe = fmmlm.Plan(w["d"], w["eps"], w["x"], w["y"], w["z"], w["layer"], p=10, leaf_cap=20)
    tab = fmmlm.Surrogate(plan=probe, tables=True)
    phi_q = probe.eval(q).cpu().numpy()
    probe.close()
    plan = fmmlm.Plan(w["d"], w["eps"], w["x"], w["y"], w["z"], w["layer"], p=10, leaf_cap=20, surrogate=tab)
    st = plan.stats()
    phi_t = plan.eval(q).cpu().numpy()
    plan.close()
    tab.close()
    out["six"] = (relerr(phi_t[t], ref), relerr(phi_q[t], ref), relerr(phi_t, phi_q))
    _say(f"  six regions p=10: tables {out['six'][0]:.3e} quadrature {out['six'][1]:.3e} "
         f"tables vs quadrature {out['six'][2]:.2e}; tasks {st['surrogate_tasks']}/{st['n_sommerfeld_tasks']} "
         f"pairs {st['surrogate_pairs']}/{st['p2p_reaction_pairs']} check {st['surrogate_check']:.2e}")
    assert st["surrogate_tasks"] == st["n_sommerfeld_tasks"]
    assert st["surrogate_pairs"] == st["p2p_reaction_pairs"]
    assert st["surrogate_check"] < 1e-10
    assert out["six"][0] < 1e-6 and out["six"][2] < 1e-9
    # three layers, p = 12: the FP64 form's 1e-7 bound holds with the tables
    w = W.config(0)
    ref = oracle_mod.potential(w["d"], w["eps"], w["x"], w["y"], w["z"], w["layer"], w["q"][0])
    probe = fmmlm.Plan(w["d"], w["eps"], w["x"], w["y"], w["z"], w["layer"], p=12, leaf_cap=40)
    tab = fmmlm.Surrogate(plan=probe, tables=True)
    probe.close()
    plan = fmmlm.Plan(w["d"], w["eps"], w["x"], w["y"], w["z"], w["layer"], p=12, leaf_cap=40, surrogate=tab)
    phi = plan.eval(torch.tensor(w["q"][0], device="cuda:0")).cpu().numpy()
    plan.close()
    tab.close()
    e = relerr(phi, ref)
    _say(f"  three layers p=12 with tables: {e:.3e}")
    assert e <= 1e-7


def test_plan_time_tables_quadrature_network():
    """Plan time of a plan with a large reaction near field (six regions, 65536 points):
    quadrature, tables (creation + plan) and the network (training + plan)."""
    from paper_1908_10863_amd import fmmlm, workloads as W
    w = W.config(4, n=65536, seed=5)
    args = (w["d"], w["eps"], w["x"], w["y"], w["z"], w["layer"])
    kw = dict(p=10, leaf_cap=128, precision=1, mac_d2=4)
    plan = fmmlm.Plan(*args, **kw)
    sq = plan.stats()
    tab = fmmlm.Surrogate(plan=plan, tables=True)
    net = fmmlm.Surrogate(plan=plan, seed=11)
    plan.close()
    rep = net.train()
    res = {"quadrature": (sq, 0.0)}
    for tag, sur, extra in (("tables", tab, tab.table_info()["seconds"]),
                            ("network", net, rep["sample_seconds"] + rep["train_seconds"])):
        pl = fmmlm.Plan(*args, surrogate=sur, **kw)
        res[tag] = (pl.stats(), extra)
        pl.close()
    for tag, (st, extra) in res.items():
        _say(f"  {tag}: creation {extra:.2f}s plan {st['plan_seconds']:.3f}s tables {st['table_seconds']:.3f}s "
             f"near field {st['nearfield_seconds']:.3f}s pairs {st['p2p_reaction_pairs']}")
    assert res["tables"][0]["nearfield_seconds"] < 0.5 * res["quadrature"][0]["nearfield_seconds"]
    tab.close()
    net.close()
