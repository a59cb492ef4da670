"""Leading term of the reaction densities (host entry point, no GPU).

sigma^{ab}_{lt,ls}(k) e^{k zinf} -> sinf as k -> infinity with remainder
O(e^{-2 k dmin}) (eq. densityasymptotic).  The library's (sinf, zinf) are
checked against the CPU oracle's dense interface solve at large k: a wrong
zinf makes sigma e^{k zinf} grow or decay exponentially in k, a wrong sinf
misses the limit.
"""
import numpy as np
import pytest

from paper_1908_10863_amd import fmmlm, workloads

MEDIA = [
    ((0.0, -1.0), (1.0, 5.0, 2.0)),
    ((0.0, -0.6, -1.4), (1.0, 3.9, 11.7, 2.5)),
    (tuple(workloads.config(4, n=12)["d"]), tuple(workloads.config(4, n=12)["eps"])),
    ((0.3,), (2.0, 7.0)),
]


def components(L):
    for lt in range(L + 1):
        for ls in range(L + 1):
            for a in (1, 2):
                for b in (1, 2):
                    if (a == 1 and lt > L - 1) or (a == 2 and lt < 1):
                        continue
                    if (b == 1 and ls > L - 1) or (b == 2 and ls < 1):
                        continue
                    yield lt, ls, a, b


@pytest.mark.parametrize("mi", range(len(MEDIA)))
def test_leading_term_matches_oracle(oracle_mod, mi):
    d, eps = MEDIA[mi]
    L = len(d)
    dmin = min([d[i - 1] - d[i] for i in range(1, L)] or [1.0])
    for lt, ls, a, b in components(L):
        si, zi = fmmlm.density_asymptotic(d, eps, lt, ls, a, b)
        idx = 2 * (a - 1) + (b - 1)
        ks = [10.0 / dmin, 15.0 / dmin]
        errs = []
        for k in ks:
            s = oracle_mod.sigma(d, eps, lt, ls, k)[idx] * np.exp(k * zi)
            errs.append(abs(s - si))
        # remainder ~ C e^{-2 k dmin}; allow the oracle's rounding on top
        assert errs[1] <= 1e-10 * max(1.0, abs(si)) + 1e-12, (lt, ls, a, b, si, errs)
        if L == 1:
            assert errs[0] < 1e-14 and zi == 0.0


def test_invalid_component_rejected():
    with pytest.raises(ValueError):
        fmmlm.density_asymptotic((0.0, -1.0), (1.0, 5.0, 2.0), 0, 0, 2, 1)
