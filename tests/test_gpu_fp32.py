"""GPU parity of the FP32 form (P2P and M2L in FP32 with compensated sums; FP64
Sommerfeld tables, normalisations, reaction operators and the top tree levels)
against the FP64 oracle: relative L2 error <= 1e-5, the stated bar of this form."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


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


def _say(m):
    print(m, flush=True)
    sys.stdout.flush()


def relerr(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _phi(F, w, dev, precision, p, cap, mac, top=3):
    import torch
    plan = F.Plan(w["d"], w["eps"], w["x"], w["y"], w["z"], w["layer"], p=p, leaf_cap=cap,
                  precision=precision, mac_d2=mac, fp64_top_levels=top)
    q = torch.tensor(w["q"][0], dtype=torch.float64, device=dev)
    out = plan.eval(q).cpu().numpy()
    plan.close()
    return out


@pytest.mark.parametrize("mac", [4, 6])
def test_fp32_small_vs_oracle(dev, F, oracle_mod, mac):
    from paper_1908_10863_amd import workloads as W
    _say(f"fp32 small mac={mac}")
    w = W.config(0, n=3000)
    ref = oracle_mod.potential(w["d"], w["eps"], w["x"], w["y"], w["z"], w["layer"], w["q"][0])
    # top-level count 0 puts every M2L level in FP32
    e32 = relerr(_phi(F, w, dev, F.FMMLM_FP32_COMPENSATED, 10, 32, mac, top=0), ref)
    e64 = relerr(_phi(F, w, dev, F.FMMLM_FP64, 10, 32, mac), ref)
    _say(f"  fp32 {e32:.3e} fp64 {e64:.3e}")
    assert e32 <= 1e-5
    # FP32 rounding adds little on top of the truncation error
    assert e32 <= e64 + 2e-6


def test_fp32_across_orders(dev, F, oracle_mod):
    """p = 4, 8, 14, 16 (other padded operator sizes than p = 10's): the FP32 form
    follows the FP64 form's truncation error down to its own rounding floor
    (about 3e-7)."""
    from paper_1908_10863_amd import workloads as W
    w = W.config(0, n=3000)
    ref = oracle_mod.potential(w["d"], w["eps"], w["x"], w["y"], w["z"], w["layer"], w["q"][0])
    for p in (4, 8, 14, 16):
        e32 = relerr(_phi(F, w, dev, F.FMMLM_FP32_COMPENSATED, p, 32, 6), ref)
        e64 = relerr(_phi(F, w, dev, F.FMMLM_FP64, p, 32, 6), ref)
        _say(f"  p {p}: fp32 {e32:.2e} fp64 {e64:.2e}")
        assert e32 <= max(1.2 * e64, 5e-7)


def test_fp32_four_million_points(dev, F, oracle_mod):
    """Four times the benchmark's size (N = 4194304, FP32 form, the benchmark's p,
    MAC and leaf cap): 24 sampled targets against the direct sum over all sources."""
    import torch
    from paper_1908_10863_amd import workloads as W
    n = 4194304
    _say(f"fp32 N={n}")
    w = W.config(2, n=n, seed=51)
    pl = F.Plan(w["d"], w["eps"], w["x"], w["y"], w["z"], w["layer"], p=10, leaf_cap=192,
                precision=F.FMMLM_FP32_COMPENSATED, mac_d2=4)
    phi = pl.eval(torch.tensor(w["q"][0], device=dev)).cpu().numpy()
    pl.close()
    t = np.sort(np.random.default_rng(52).choice(n, 24, replace=False))
    ref = oracle_mod.potential(w["d"], w["eps"], w["x"], w["y"], w["z"], w["layer"], w["q"][0], targets=t)
    e = relerr(phi[t], ref)
    _say(f"  rel L2 {e:.2e}")
    assert e <= 1e-5


def test_single_interface_fp32_and_batched(dev, F, oracle_mod):
    """One interface (two half-spaces, eps 2 and 9): the FP32 form and the batched
    FP32 form (three vectors, batched kernels forced) against the quadrature direct
    sum, <= 1e-5; the batched result is linear in the charges."""
    import torch
    rng = np.random.default_rng(91)
    d, eps = [0.0], [2.0, 9.0]
    n = 3000
    lay = np.repeat([0, 1], n // 2).astype(np.int32)
    z = np.where(lay == 0, rng.uniform(0.05, 1.0, n), rng.uniform(-1.0, -0.05, n))
    x, y, q = rng.uniform(-0.5, 0.5, n), rng.uniform(-0.5, 0.5, n), rng.uniform(-1, 1, n)
    ref = oracle_mod.potential(d, eps, x, y, z, lay, q, method="quad")
    qt = torch.tensor(q, device=dev)
    pl = F.Plan(d, eps, x, y, z, lay, p=10, leaf_cap=32, precision=1, mac_d2=4)
    e = relerr(pl.eval(qt).cpu().numpy(), ref)
    pl.close()
    pl = F.Plan(d, eps, x, y, z, lay, p=10, leaf_cap=32, precision=1, mac_d2=4, max_rhs=8)
    pl.set_variants(batch_min=2)
    phi = pl.eval(torch.stack([qt, -qt, 2 * qt])).cpu().numpy()
    pl.close()
    eb = relerr(phi[0], ref)
    _say(f"  one interface: fp32 {e:.2e} batched {eb:.2e}")
    assert e <= 1e-5 and eb <= 1e-5
    assert relerr(phi[2], 2 * phi[0]) < 1e-6 and relerr(-phi[1], phi[0]) < 1e-6


def test_fp32_six_region_medium(dev, F, oracle_mod):
    """The six-region medium (five interfaces, about 100 reaction components, the
    FP32 form's sparse top levels and reaction chunks all in play) against the
    quadrature direct sum on 48 targets: FP32 form <= 1e-5, FP64 form <= 1e-6."""
    from paper_1908_10863_amd import workloads as W
    _say("fp32 six regions")
    w = W.config(4, n=12000, seed=44)
    t = np.sort(np.random.default_rng(45).choice(12000, 48, replace=False))
    ref = oracle_mod.potential(w["d"], w["eps"], w["x"], w["y"], w["z"], w["layer"], w["q"][0], targets=t,
                               method="quad")
    e32 = relerr(_phi(F, w, dev, F.FMMLM_FP32_COMPENSATED, 10, 64, 4)[t], ref)
    e64 = relerr(_phi(F, w, dev, F.FMMLM_FP64, 10, 64, 6)[t], ref)
    _say(f"  fp32 {e32:.3e} fp64 {e64:.3e}")
    assert e32 <= 1e-5
    assert e64 <= 1e-6


def test_fp32_full_size_sampled(dev, F, oracle_mod):
    """Workload 3 at full size (N = 1048576, p = 10): 64 sampled targets against the
    direct sum over all sources."""
    from paper_1908_10863_amd import workloads as W
    _say("fp32 full size")
    w = W.config(2)
    rng = np.random.default_rng(321)
    t = np.sort(rng.choice(len(w["x"]), 64, replace=False))
    ref = oracle_mod.potential(w["d"], w["eps"], w["x"], w["y"], w["z"], w["layer"], w["q"][0], targets=t)
    for mac in (4, 6):
        phi = _phi(F, w, dev, F.FMMLM_FP32_COMPENSATED, 10, 128, mac)
        e = relerr(phi[t], ref)
        _say(f"  mac={mac} rel L2 {e:.3e}")
        assert e <= 1e-5


@pytest.mark.parametrize("precision", [0, 1])
def test_m2l_operator_groups(dev, F, oracle_mod, precision):
    """Below the top levels the M2L runs in chunks of up to four operators that reach the
    same targets, one step per operator and one partial per target for all of a chunk's
    steps.  On a uniform workload with interior boxes most pairs are grouped (fewer
    chunks than steps, at most four steps a chunk), every pair sits in one step column
    (steps x columns >= pairs below the top levels), and the result meets the 1e-5 bar
    against the direct sum on sampled targets in both forms."""
    import torch
    from paper_1908_10863_amd import workloads as W
    _say(f"M2L operator groups, precision={precision}")
    w = W.config(2, n=200000, seed=5)
    plan = F.Plan(w["d"], w["eps"], w["x"], w["y"], w["z"], w["layer"], p=10, leaf_cap=64,
                  precision=precision, mac_d2=4)
    st = plan.stats()
    pairs = st["m2l_free_pairs"] + st["m2l_reaction_pairs"] - st["m2l_top_pairs"]
    _say(f"  chunks {st['m2l_chunks']} steps {st['m2l_steps']} pairs {pairs}")
    assert 0 < st["m2l_chunks"] < st["m2l_steps"] <= 4 * st["m2l_chunks"]
    assert st["m2l_steps"] >= 1.5 * st["m2l_chunks"]  # most pairs grouped
    assert pairs <= st["m2l_steps"] * st["m2l_tile_cols"]
    q = torch.tensor(w["q"][0], dtype=torch.float64, device=dev)
    phi = plan.eval(q).cpu().numpy()
    plan.close()
    t = np.sort(np.random.default_rng(55).choice(len(w["x"]), 128, replace=False))
    ref = oracle_mod.potential(w["d"], w["eps"], w["x"], w["y"], w["z"], w["layer"], w["q"][0], targets=t)
    e = relerr(phi[t], ref)
    _say(f"  rel L2 {e:.3e}")
    assert e <= 1e-5


@pytest.mark.parametrize("precision", [0, 1])
def test_streams_and_tuning_do_not_change_results(dev, F, precision):
    """An unprofiled evaluation runs the near field and the sparse top levels on
    their own streams, with part of the free P2P after the main M2L and extra LDS
    reserved by the P2P launch; a profiled one runs every stage in order on one
    stream.  Each kernel's arithmetic is the same, so the results are bit-equal,
    and so are those of every M2L tile shape (set_variants)."""
    import torch
    from paper_1908_10863_amd import workloads as W
    _say(f"overlapped == profiled, precision={precision}")
    w = W.config(2, n=60000, seed=21)
    plan = F.Plan(w["d"], w["eps"], w["x"], w["y"], w["z"], w["layer"], p=10, leaf_cap=96,
                  precision=precision, mac_d2=4)
    st = plan.stats()
    if precision == 1:
        assert st["p2p_split_pct"] in (0, 25, 50, 75, 100)
        assert all(t > 0 for t in st["p2p_split_ms"])
        assert st["m2l_variant"] == int(np.argmin(st["m2l_eval_ms"]))
    q = torch.tensor(w["q"][0], dtype=torch.float64, device=dev)
    a = plan.eval(q).cpu().numpy()
    plan.profile_begin(1)
    b = plan.eval(q).cpu().numpy()
    stages, n = plan.profile_end()
    assert n == 1
    assert np.array_equal(a, b)
    if precision == 1:
        for v in range(6):
            plan.set_variants(m2l=v)
            assert np.array_equal(plan.eval(q).cpu().numpy(), a), v
    plan.close()
