"""Graph mode: an evaluation captured into a HIP graph and replayed.

The plan captures its launch sequence on the first call on a side stream and
replays it while the arguments stay the same.  Each replay follows eager work
(new charges written into the same tensor, a synchronisation) and must equal,
bit for bit, the same plan's eager evaluation (null stream) of those charges:
FP64 and FP32 forms, one vector and a batch of three.  Changing the output
buffer captures anew.
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


@pytest.mark.parametrize("precision,nrhs", [(0, 1), (1, 1), (1, 3)])
def test_graph_replays_equal_eager(F, precision, nrhs):
    import torch
    from paper_1908_10863_amd import workloads as W
    _say(f"graph mode precision={precision} nrhs={nrhs}")
    w = W.config(0, n=1200)
    plan = F.Plan(w["d"], w["eps"], w["x"], w["y"], w["z"], w["layer"], p=8, leaf_cap=40,
                  precision=precision, max_rhs=nrhs, graph=True)
    plan.set_variants(batch_min=2)
    side = torch.cuda.Stream()
    rng = np.random.default_rng(5)
    shape = (nrhs, 1200) if nrhs > 1 else (1200,)
    q = torch.zeros(shape, dtype=torch.float64, device="cuda:0")
    out = torch.zeros_like(q)
    for it in range(4):
        q.copy_(torch.tensor(rng.uniform(-1, 1, shape), device="cuda:0"))
        torch.cuda.synchronize()
        ref = plan.eval(q, stream=torch.cuda.default_stream()).cpu().numpy()  # eager
        side.wait_stream(torch.cuda.current_stream())
        plan.eval(q, out=out, stream=side)  # capture on it == 0, replay after
        side.synchronize()
        got = out.cpu().numpy()
        assert np.array_equal(got, ref), f"replay {it}"
    # another output buffer: captured anew, same values
    out2 = torch.zeros_like(q)
    plan.eval(q, out=out2, stream=side)
    side.synchronize()
    assert np.array_equal(out2.cpu().numpy(), ref)
    plan.close()
