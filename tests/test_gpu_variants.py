"""Every kernel variant the autotuners choose from gives the tuned variant's result.

The FP32 M2L has six tile shapes and the batched FP32 M2L five shapes, each as
one block per target box and as a persistent XCD-aware grid.  They take the
same sums in the same order per output element, so each variant must match the
variant the plan's autotuner picked, bit for bit; the tuned result itself is
checked against the direct-sum oracle.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def F():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1908_10863_amd import fmmlm
    fmmlm.lib()
    return fmmlm


def test_fp32_m2l_shapes(F, oracle_mod):
    import torch
    from paper_1908_10863_amd import workloads as W
    w = W.config(0, n=3000, seed=9)
    plan = F.Plan(w["d"], w["eps"], w["x"], w["y"], w["z"], w["layer"], p=10, leaf_cap=24, precision=1,
                  mac_d2=4)
    st = plan.stats()
    _say(f"FP32 M2L tuned variant {st['m2l_variant']} times {[round(t, 4) for t in st['m2l_variant_ms']]}")
    q = torch.tensor(w["q"][0], device="cuda:0")
    ref = plan.eval(q).cpu().numpy()
    t = np.arange(0, 3000, 15)
    orc = oracle_mod.potential(w["d"], w["eps"], w["x"], w["y"], w["z"], w["layer"], w["q"][0], targets=t,
                               method="image3")
    assert np.linalg.norm(ref[t] - orc) / np.linalg.norm(orc) < 1e-5
    for v in range(6):
        plan.set_variants(m2l=v)
        got = plan.eval(q).cpu().numpy()
        assert np.array_equal(got, ref), f"variant {v}"
    with pytest.raises(ValueError):
        plan.set_variants(m2l=6)
    plan.close()


def test_batched_m2l_variants(F, oracle_mod):
    import torch
    from paper_1908_10863_amd import workloads as W
    w = W.config(0, n=3000, seed=10)
    g = 64
    plan = F.Plan(w["d"], w["eps"], w["x"], w["y"], w["z"], w["layer"], p=10, leaf_cap=24, precision=1,
                  mac_d2=4, max_rhs=g)
    plan.set_variants(batch_min=2)
    st = plan.stats()
    _say(f"batched M2L tuned variant {st['batch_variant']} times "
         f"{[round(t, 4) for t in st['batch_variant_ms']]}")
    rng = np.random.default_rng(3)
    Q = torch.tensor(rng.uniform(-1, 1, (g, 3000)), device="cuda:0")
    ref = plan.eval(Q).cpu().numpy()
    t = np.arange(0, 3000, 30)
    orc = oracle_mod.potential(w["d"], w["eps"], w["x"], w["y"], w["z"], w["layer"],
                               Q[5].cpu().numpy(), targets=t, method="image3")
    assert np.linalg.norm(ref[5, t] - orc) / np.linalg.norm(orc) < 1e-5
    for v in range(10):
        plan.set_variants(batch=v)
        got = plan.eval(Q).cpu().numpy()
        assert np.array_equal(got, ref), f"variant {v}"
    with pytest.raises(ValueError):
        plan.set_variants(batch=10)
    plan.close()
