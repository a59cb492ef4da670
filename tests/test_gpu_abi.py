"""C-ABI error paths and pointer kinds that need a plan (so a GPU): evaluation argument
checks, geometry passed as device pointers, and overlap detection (FMMLM_EBUSY)."""
import ctypes
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def small():
    from paper_1908_10863_amd import fmmlm, workloads
    w = workloads.config(0, n=900)
    plan = fmmlm.Plan(w["d"], w["eps"], w["x"], w["y"], w["z"], w["layer"], p=6, leaf_cap=40, max_rhs=2)
    yield fmmlm, w, plan
    plan.close()


def _eval_rc(fmmlm, plan, nrhs, q, ldq, phi, ldphi, parts):
    return fmmlm.lib().fmm_layered_eval(plan._h, nrhs, None if q is None else ctypes.c_void_p(q.data_ptr()), ldq,
                                        None if phi is None else ctypes.c_void_p(phi.data_ptr()), ldphi, parts,
                                        None)


def test_eval_argument_errors(small):
    import torch
    fmmlm, w, plan = small
    n = len(w["x"])
    _say(f"eval argument errors n={n}")
    q = torch.zeros((3, n + 4), dtype=torch.float64, device="cuda")
    phi = torch.zeros_like(q)
    both = fmmlm.FREE | fmmlm.REACTION
    assert _eval_rc(fmmlm, plan, 3, q, n + 4, phi, n + 4, both) == -1      # nrhs > max_rhs = 2
    assert _eval_rc(fmmlm, plan, 0, q, n + 4, phi, n + 4, both) == -1      # nrhs < 1
    assert _eval_rc(fmmlm, plan, 1, q, n - 1, phi, n + 4, both) == -1      # ldq < n
    assert _eval_rc(fmmlm, plan, 1, q, n + 4, phi, n - 1, both) == -1      # ldphi < n
    assert _eval_rc(fmmlm, plan, 1, q, n, phi, n, 0) == -1                 # no part
    assert _eval_rc(fmmlm, plan, 1, q, n, phi, n, 4) == -1                 # unknown part bit
    assert _eval_rc(fmmlm, plan, 1, None, n, phi, n, both) == -1           # null charges
    assert _eval_rc(fmmlm, plan, 1, q, n, None, n, both) == -1             # null potentials
    # a padded leading dimension is accepted and gives the same potentials
    qq = torch.tensor(w["q"][0], device="cuda")
    ref = plan.eval(qq).cpu().numpy()
    q[0, :n] = qq
    q[1, :n] = 2.0 * qq
    assert _eval_rc(fmmlm, plan, 2, q, n + 4, phi, n + 4, both) == 0
    torch.cuda.synchronize()
    np.testing.assert_allclose(phi[0, :n].cpu().numpy(), ref, rtol=1e-13, atol=0)
    np.testing.assert_allclose(phi[1, :n].cpu().numpy(), 2.0 * ref, rtol=1e-13, atol=0)


def test_geometry_from_device_pointers(small):
    """The plan copies geometry from device pointers as from host ones: the same plan."""
    import torch
    fmmlm, w, plan = small
    L = fmmlm.lib()
    _say("geometry from device pointers")
    t = {k: torch.tensor(np.ascontiguousarray(w[k]), device="cuda") for k in ("d", "eps", "x", "y", "z")}
    lay = torch.tensor(np.ascontiguousarray(w["layer"], np.int32), device="cuda")
    o = fmmlm.Opts()
    L.fmmlm_default_opts(ctypes.byref(o))
    o.leaf_cap = 40
    o.max_rhs = 2
    h = ctypes.c_void_p()
    vp = lambda a: ctypes.c_void_p(a.data_ptr())  # noqa: E731
    rc = L.fmm_layered_plan(len(w["d"]), vp(t["d"]), vp(t["eps"]), len(w["x"]), vp(t["x"]), vp(t["y"]),
                            vp(t["z"]), vp(lay), 6, ctypes.byref(o), None, ctypes.byref(h))
    assert rc == 0
    try:
        q = torch.tensor(w["q"][0], device="cuda")
        phi = torch.empty_like(q)
        assert L.fmm_layered_eval(h, 1, vp(q), len(q), vp(phi), len(q), 3, None) == 0
        torch.cuda.synchronize()
        ref = plan.eval(q).cpu().numpy()
        np.testing.assert_array_equal(phi.cpu().numpy(), ref)
        s1, s2 = fmmlm.Stats(), fmmlm.Stats()
        L.fmm_layered_plan_stats(h, ctypes.byref(s1))
        L.fmm_layered_plan_stats(plan._h, ctypes.byref(s2))
        assert (s1.n_boxes, s1.m2l_free_pairs, s1.p2p_free_pairs) == (s2.n_boxes, s2.m2l_free_pairs,
                                                                     s2.p2p_free_pairs)
    finally:
        L.fmm_layered_destroy(h)


def test_overlapping_evaluations_are_refused(small):
    """An evaluation on stream B while the plan's last evaluation on stream A is still
    queued behind a long spin (torch's bounded sleep kernel) is refused with EBUSY; after
    A drains, or on the same stream, it runs."""
    import torch
    fmmlm, w, plan = small
    _say("overlap detection")
    q = torch.tensor(w["q"][0], device="cuda")
    out_a = torch.empty_like(q)
    out_b = torch.empty_like(q)
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    ref = plan.eval(q).cpu().numpy()
    with torch.cuda.stream(sa):
        torch.cuda._sleep(200_000_000)            # about 0.1 s of spinning on stream A
        plan.eval(q, out=out_a, stream=sa)
        plan.eval(q, out=out_a, stream=sa)        # same stream: ordered, accepted
    with pytest.raises(RuntimeError, match="in use"):
        plan.eval(q, out=out_b, stream=sb)
    sa.synchronize()
    plan.eval(q, out=out_b, stream=sb)            # A has finished: accepted
    sb.synchronize()
    np.testing.assert_array_equal(out_a.cpu().numpy(), ref)
    np.testing.assert_array_equal(out_b.cpu().numpy(), ref)
    # the solve checks the same way
    with torch.cuda.stream(sa):
        torch.cuda._sleep(200_000_000)
        plan.eval(q, out=out_a, stream=sa)
    with pytest.raises(RuntimeError, match="in use"):
        plan.solve(q, stream=sb, max_iters=2)
    torch.cuda.synchronize()
