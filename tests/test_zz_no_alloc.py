"""The allocation-free Sommerfeld entry point (fmm_layered_sommerfeld_noalloc) against
fmm_layered_sommerfeld on the same points, through the C ABI: two calls in a row, the
second with fewer points (the staging array keeps the first call's contents), plus the
size limit and the invalid-point marking."""
import ctypes

import numpy as np
import pytest

D3 = [0.0, -1.0]
E3 = [1.0, 5.0, 2.0]
D4 = [0.0, -0.6, -1.4]
E4 = [1.0, 3.9, 11.7, 2.5]


def _points(n, seed, S):
    rng = np.random.default_rng(seed)
    # rho on the M2L lattice (0 or >= 2 box sizes: the recurrence's range) and free z
    rho = S * np.where(rng.random(n) < 0.2, 0.0, rng.uniform(2.0, 8.0, n))
    z = rng.uniform(0.2, 2.5, n)
    return rho, z


@pytest.mark.gpu
@pytest.mark.parametrize("medium,comp,npts", [((D3, E3), (1, 1, 1, 1), (3000, 700)),
                                              ((D4, E4), (2, 0, 2, 1), (1500, 257))])
def test_noalloc_matches_allocating_entry(medium, comp, npts):
    import torch
    from paper_1908_10863_amd import fmmlm
    d, eps = medium
    S, nmax = 0.25, 20
    nc = (nmax + 1) * (nmax + 2) // 2
    for call, n in enumerate(npts):
        print(f"noalloc call {call}: medium L={len(d)} comp={comp} npts={n}", flush=True)
        rho, z = _points(n, 10 + call, S)
        ref = fmmlm.sommerfeld(d, eps, *comp, S, rho, z, nmax)
        out = torch.full((n, nc), 7.0, dtype=torch.float64, device="cuda")
        fmmlm.sommerfeld_noalloc(d, eps, *comp, S, torch.tensor(rho, device="cuda"),
                                 torch.tensor(z, device="cuda"), nmax, out)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        # the same kernel on the same tasks: bit-equal
        np.testing.assert_array_equal(got, ref)


@pytest.mark.gpu
def test_noalloc_limits_and_invalid_points():
    import torch
    from paper_1908_10863_amd import fmmlm
    L = fmmlm.lib()
    nmax, S = 6, 0.5
    nc = (nmax + 1) * (nmax + 2) // 2
    big = 65537
    rho = torch.zeros(big, dtype=torch.float64, device="cuda")
    z = torch.ones(big, dtype=torch.float64, device="cuda")
    out = torch.zeros((big, nc), dtype=torch.float64, device="cuda")
    d = np.asarray(D3)
    e = np.asarray(E3)
    rc = L.fmm_layered_sommerfeld_noalloc(2, ctypes.c_void_p(d.ctypes.data), ctypes.c_void_p(e.ctypes.data),
                                          1, 1, 1, 1, S, big, ctypes.c_void_p(rho.data_ptr()),
                                          ctypes.c_void_p(z.data_ptr()), nmax, ctypes.c_void_p(out.data_ptr()),
                                          None)
    assert rc == -1
    assert L.fmm_layered_sommerfeld_noalloc(2, ctypes.c_void_p(d.ctypes.data), ctypes.c_void_p(e.ctypes.data),
                                            1, 1, 1, 1, S, 0, ctypes.c_void_p(rho.data_ptr()),
                                            ctypes.c_void_p(z.data_ptr()), nmax, ctypes.c_void_p(out.data_ptr()),
                                            None) == -1
    # points 1 and 3 are invalid (negative rho, z = 0): NaN there, the others as the allocating entry
    r = np.array([0.0, -1.0, 1.5, 2.0, 3.0])
    zz = np.array([0.4, 0.5, 0.6, 0.0, 1.1])
    o = torch.zeros((5, nc), dtype=torch.float64, device="cuda")
    fmmlm.sommerfeld_noalloc(D3, E3, 1, 1, 1, 1, S, torch.tensor(r, device="cuda"), torch.tensor(zz, device="cuda"),
                             nmax, o)
    torch.cuda.synchronize()
    got = o.cpu().numpy()
    assert np.all(np.isnan(got[[1, 3]]))
    ok = [0, 2, 4]
    ref = fmmlm.sommerfeld(D3, E3, 1, 1, 1, 1, S, r[ok], zz[ok], nmax)
    np.testing.assert_array_equal(got[ok], ref)
