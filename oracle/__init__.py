"""Oracle -- TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously-correct CPU references for what the layered-media FMM
computes (Wang, Zhang & Cai, arXiv:1908.10863).  Only ``tests/``,
``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may import
this package.  It shares no code with the GPU path (``paper_1908_10863_amd``)
and never imports it.

Contents and the passage each follows:

* ``sigma``            reaction densities sigma^{ab}_{l l'}(k) by a direct solve of
                        the interface system (App. A, interface conditions).
* ``sigma_ab``, ``potential_ab``  the same for general interface conditions
                        a u and b du/dz continuous (App. A's general
                        conditions; classic a = 1, b = eps), direct solve.
* ``sigma3``           the explicit three-layer densities (App. A,
                        eqs. densitythreelayer1-3, with the two readings listed
                        in the design notes).
* ``reaction_quad``    one reaction component, eq. generalcomponents reduced to
                        1/(4 pi) int J0(k rho) e^{-k zeta} sigma(k) dk, by fixed
                        composite Gauss-Legendre quadrature.
* ``reaction_image3``  the same kernel for three layers as an image series.
* ``potential``        direct O(N * targets) sum of eq. totalinteraction.
* ``matrix``           the same pair values as a dense N x N matrix.
* ``solve_dense``      the solution of (diag + G) x = b by a dense LU solve: what
                        an iterative solve around the FMM matvec computes (Sec. 1).
* ``sommerfeld_sigma1`` closed form of S^n I_nm for sigma == 1 (Sec. 3.4, the
                        identity used for Table 3.1).
* ``sommerfeld_image3`` S^n I_nm for a three-layer density: image series of the
                        sigma == 1 closed form.
* ``sommerfeld_mp``    S^n I_nm by 30-digit mpmath quadrature of
                        eq. scaledsommerfeldint, any number of layers.
* ``morton_sort``      the octree's key definition and stable sort.
* ``polarization_z``   equivalent polarization source heights (eq. eqpolarizedsource).
* ``mlp``              (submodule) the surrogate network of the learned form:
                        forward pass, loss, chain-rule gradient, Adam step.

Pins for every function are in tests/test_oracle_*.py.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so (gcc, -O2, OpenMP, no FMA contraction)."""
    src = os.path.join(_HERE, "oracle.c")
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(src):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
               "-o", tmp, src, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int32)
        lp = ctypes.POINTER(ctypes.c_int64)
        lib.oracle_sigma.argtypes = [ctypes.c_int, dp, dp, ctypes.c_int, ctypes.c_int,
                                     ctypes.c_double, dp]
        lib.oracle_sigma.restype = ctypes.c_int
        lib.oracle_sigma3.argtypes = [dp, dp, ctypes.c_int, ctypes.c_int, ctypes.c_double, dp]
        lib.oracle_sigma3.restype = ctypes.c_int
        lib.oracle_image3_terms.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                            ctypes.c_int, ctypes.c_int, dp,
                                            ctypes.POINTER(ctypes.c_int)]
        lib.oracle_image3_terms.restype = ctypes.c_int
        lib.oracle_reaction_quad.argtypes = [ctypes.c_int, dp, dp, ctypes.c_int, ctypes.c_int,
                                             ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                             ctypes.c_double]
        lib.oracle_reaction_quad.restype = ctypes.c_double
        lib.oracle_reaction_image3.argtypes = [dp, dp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                               ctypes.c_int, ctypes.c_double, ctypes.c_double]
        lib.oracle_reaction_image3.restype = ctypes.c_double
        lib.oracle_potential.argtypes = [ctypes.c_int, dp, dp, ctypes.c_int64, dp, dp, dp, ip,
                                         dp, ctypes.c_int64, lp, ctypes.c_int, ctypes.c_int, dp]
        lib.oracle_potential.restype = ctypes.c_int
        lib.oracle_matrix.argtypes = [ctypes.c_int, dp, dp, ctypes.c_int64, dp, dp, dp, ip,
                                      ctypes.c_int64, lp, ctypes.c_int, ctypes.c_int, dp, dp]
        lib.oracle_matrix.restype = ctypes.c_int
        lib.oracle_sigma_ab.argtypes = [ctypes.c_int, dp, dp, dp, ctypes.c_int, ctypes.c_int,
                                        ctypes.c_double, dp]
        lib.oracle_sigma_ab.restype = ctypes.c_int
        lib.oracle_potential_ab.argtypes = [ctypes.c_int, dp, dp, dp, ctypes.c_int64, dp, dp, dp, ip,
                                            dp, ctypes.c_int64, lp, ctypes.c_int, dp]
        lib.oracle_potential_ab.restype = ctypes.c_int
        lib.oracle_num_threads.argtypes = []
        lib.oracle_num_threads.restype = ctypes.c_int
        lib.oracle_set_threads.argtypes = [ctypes.c_int]
        lib.oracle_set_threads.restype = None
        _lib = lib
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of the oracle's later parallel loops (OpenMP)."""
    _load().oracle_set_threads(int(n))


# --------------------------------------------------------------------------
# reaction densities
# --------------------------------------------------------------------------
def sigma(d, eps, lt: int, ls: int, k: float) -> np.ndarray:
    """sigma^{ab}_{lt,ls}(k) for a,b in {1,2}, indexed [2(a-1)+(b-1)]; invalid -> 0."""
    d = _f64(d)
    eps = _f64(eps)
    out = np.zeros(4)
    rc = _load().oracle_sigma(len(d), _dp(d), _dp(eps), lt, ls, float(k), _dp(out))
    if rc:
        raise ValueError(f"oracle_sigma failed ({rc})")
    return out


def sigma_ab(d, a, b, lt: int, ls: int, k: float) -> np.ndarray:
    """sigma^{ab}_{lt,ls}(k) for the general interface conditions of App. A,
    a_{i-1} u_{i-1} = a_i u_i and b_{i-1} u'_{i-1} = b_i u'_i at every interface
    (classic: a = 1, b = eps), by the same direct solve; indexed like sigma."""
    d = _f64(d)
    a = _f64(a)
    b = _f64(b)
    out = np.zeros(4)
    rc = _load().oracle_sigma_ab(len(d), _dp(d), _dp(a), _dp(b), int(lt), int(ls), float(k), _dp(out))
    if rc:
        raise ValueError(f"oracle_sigma_ab failed ({rc})")
    return out


def potential_ab(d, a, b, x, y, z, layer, q, targets=None, parts=3) -> np.ndarray:
    """Direct sum of eq. totalinteraction for the general interface conditions
    (coefficients a, b), reaction kernels by quadrature."""
    d, a, b = _f64(d), _f64(a), _f64(b)
    x, y, z, q = _f64(x), _f64(y), _f64(z), _f64(q)
    layer = np.ascontiguousarray(np.asarray(layer, dtype=np.int32))
    n = len(x)
    if targets is None:
        targets = np.arange(n, dtype=np.int64)
    targets = np.ascontiguousarray(np.asarray(targets, dtype=np.int64))
    out = np.zeros(len(targets))
    rc = _load().oracle_potential_ab(len(d), _dp(d), _dp(a), _dp(b), n, _dp(x), _dp(y), _dp(z),
                                     layer.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _dp(q),
                                     len(targets), targets.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                     int(parts), _dp(out))
    if rc:
        raise ValueError(f"oracle_potential_ab failed ({rc})")
    return out


def sigma3(d, eps, lt: int, ls: int, k: float) -> np.ndarray:
    d = _f64(d)
    eps = _f64(eps)
    assert len(d) == 2 and len(eps) == 3
    out = np.zeros(4)
    _load().oracle_sigma3(_dp(d), _dp(eps), lt, ls, float(k), _dp(out))
    return out


def image3_terms(eps, lt, ls, a, b, maxterm=1200):
    eps = _f64(eps)
    coef = np.zeros(maxterm)
    shift = np.zeros(maxterm, dtype=np.int32)
    n = _load().oracle_image3_terms(_dp(eps), lt, ls, a, b, maxterm, _dp(coef),
                                    shift.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
    return coef[:n].copy(), shift[:n].copy()


def valid(L: int, layer: int, side: int) -> bool:
    return layer <= L - 1 if side == 1 else layer >= 1


def reaction_quad(d, eps, lt, ls, a, b, rho, zeta) -> float:
    """u^{ab}_{lt ls} = 1/(4pi) int_0^inf J0(k rho) e^{-k zeta} sigma^{ab}(k) dk.

    ``d=[]`` means sigma == 1 (the free-space Sommerfeld identity)."""
    d = _f64(d)
    eps = _f64(eps) if len(d) else np.ones(1)
    return float(_load().oracle_reaction_quad(len(d), _dp(d), _dp(eps), lt, ls, a, b,
                                              float(rho), float(zeta)))


def reaction_image3(d, eps, lt, ls, a, b, rho, zeta) -> float:
    d = _f64(d)
    eps = _f64(eps)
    return float(_load().oracle_reaction_image3(_dp(d), _dp(eps), lt, ls, a, b,
                                                float(rho), float(zeta)))


def zeta_of(d, lt, ls, a, b, z, zs) -> float:
    """Exponent of eq. zexponential: interface-relative target + source distances."""
    t = (z - d[lt]) if a == 1 else (d[lt - 1] - z)
    s = (zs - d[ls]) if b == 1 else (d[ls - 1] - zs)
    return t + s


def potential(d, eps, x, y, z, layer, q, targets=None, method="auto", parts=3) -> np.ndarray:
    """Direct sum of eq. totalinteraction at the selected targets.

    parts: 1 free space (j != i, same layer), 2 reaction (all j incl. j == i), 3 both.
    method: 'quad' (any L), 'image3' (three layers), 'table' (any L: the quadrature's kernel
    tabulated per component and interpolated, certified against the quadrature at random
    points to 1e-12 of the component's largest value; for sums too large for 'quad'),
    'auto' (image3 when L == 2)."""
    d = _f64(d)
    eps = _f64(eps)
    x, y, z, q = _f64(x), _f64(y), _f64(z), _f64(q)
    layer = np.ascontiguousarray(np.asarray(layer, dtype=np.int32))
    n = len(x)
    if targets is None:
        targets = np.arange(n, dtype=np.int64)
    targets = np.ascontiguousarray(np.asarray(targets, dtype=np.int64))
    if method == "auto":
        method = "image3" if len(d) == 2 else "quad"
    m = {"quad": 0, "image3": 1, "table": 2}[method]
    out = np.zeros(len(targets))
    rc = _load().oracle_potential(len(d), _dp(d), _dp(eps), n, _dp(x), _dp(y), _dp(z),
                                  layer.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _dp(q),
                                  len(targets),
                                  targets.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                  m, int(parts), _dp(out))
    if rc == -5:
        raise ValueError("oracle_potential: the tabulated kernels could not be certified for this geometry")
    if rc:
        raise ValueError(f"oracle_potential failed ({rc})")
    return out


def matrix(d, eps, x, y, z, layer, method="auto", parts=3) -> np.ndarray:
    """The dense N x N matrix of eq. totalinteraction: G[i, j] is the potential at
    point i of a unit charge at point j (free part for j != i in the same layer,
    reaction part for every j), so that G @ q == potential(q)."""
    d = _f64(d)
    eps = _f64(eps)
    x, y, z = _f64(x), _f64(y), _f64(z)
    layer = np.ascontiguousarray(np.asarray(layer, dtype=np.int32))
    n = len(x)
    targets = np.arange(n, dtype=np.int64)
    if method == "auto":
        method = "image3" if len(d) == 2 else "quad"
    m = {"quad": 0, "image3": 1}[method]
    G = np.zeros((n, n))
    scratch = np.zeros(n)
    rc = _load().oracle_matrix(len(d), _dp(d), _dp(eps), n, _dp(x), _dp(y), _dp(z),
                               layer.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), n,
                               targets.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), m, int(parts),
                               _dp(scratch), _dp(G))
    if rc:
        raise ValueError(f"oracle_matrix failed ({rc})")
    return G


def solve_dense(G, diag, b) -> np.ndarray:
    """The solution x of the second-kind system (diag(diag) + G) x = b, the
    product whose G part the FMM evaluates (the iterative solve of the
    paper's motivating application, Sec. 1), by a dense LU solve."""
    A = np.array(G, dtype=np.float64, copy=True)
    A[np.diag_indices_from(A)] += _f64(diag)
    return np.linalg.solve(A, _f64(b))


# --------------------------------------------------------------------------
# Sommerfeld-type integrals S^n I_nm (eq. scaledsommerfeldint)
# --------------------------------------------------------------------------
def legendre_hat(n: int, m: int, x: float) -> float:
    """Normalised associated Legendre function of eq. sphericalharmonics:
    Y_n^m = Phat_n^m(cos theta) e^{i m phi}, no Condon-Shortley phase in Y."""
    from scipy.special import lpmv
    mm = abs(m)
    val = lpmv(mm, n, x)  # includes (-1)^m
    val *= (-1) ** mm * math.sqrt((2 * n + 1) / (4 * math.pi) * math.factorial(n - mm)
                                  / math.factorial(n + mm))
    if m < 0:
        val *= (-1) ** mm
    return float(val)


def sommerfeld_sigma1(n: int, m: int, rho: float, z: float, S: float) -> float:
    """S^n I_nm for sigma == 1: r^n I_nm = sqrt(4 pi/(2n+1)) Phat_n^m(z/r)/r (Sec. 3.4)."""
    r = math.hypot(rho, z)
    return (S / r) ** n * math.sqrt(4 * math.pi / (2 * n + 1)) * legendre_hat(n, m, z / r) / r


def sommerfeld_image3(d, eps, lt, ls, a, b, n, m, rho, z, S) -> float:
    """S^n I^{ab}_nm for a three-layer density: sigma = sum c_t e^{-k s_t D} turns the
    integral into sum c_t (S^n I_nm of sigma == 1 at height z + s_t D)."""
    coef, shift = image3_terms(eps, lt, ls, a, b)
    D = float(d[0] - d[1])
    tot = 0.0
    for c, s in zip(coef[::-1], shift[::-1]):
        tot += c * sommerfeld_sigma1(n, m, rho, z + s * D, S)
    return tot


def sigma_mp(d, eps, lt, ls, k, dps=30):
    """Direct interface solve in mpmath (same system as ``sigma``)."""
    import mpmath as mp
    with mp.workdps(dps):
        L = len(d)
        nn = 2 * L
        A = mp.zeros(nn, nn)
        R = mp.zeros(nn, 2)
        k = mp.mpmathify(k)

        def c1(i):
            return i

        def c2(i):
            return L + i - 1
        for i in range(L):
            ei = mp.exp(-k * (mp.mpf(d[i - 1]) - mp.mpf(d[i]))) if i >= 1 else 0
            ei1 = mp.exp(-k * (mp.mpf(d[i]) - mp.mpf(d[i + 1]))) if i + 1 <= L - 1 else 0
            rc, rf = 2 * i, 2 * i + 1
            A[rc, c1(i)] += 1
            if i >= 1:
                A[rc, c2(i)] += ei
            if i + 1 <= L - 1:
                A[rc, c1(i + 1)] -= ei1
            A[rc, c2(i + 1)] -= 1
            if ls == i:
                R[rc, 0] -= 1
            if ls == i + 1:
                R[rc, 1] += 1
            A[rf, c1(i)] += eps[i]
            if i >= 1:
                A[rf, c2(i)] -= eps[i] * ei
            if i + 1 <= L - 1:
                A[rf, c1(i + 1)] -= eps[i + 1] * ei1
            A[rf, c2(i + 1)] += eps[i + 1]
            if ls == i:
                R[rf, 0] += eps[i]
            if ls == i + 1:
                R[rf, 1] += eps[i + 1]
        X = [mp.lu_solve(A, R.column(0)), mp.lu_solve(A, R.column(1))]
        out = []
        for a in (1, 2):
            for b in (1, 2):
                if valid(L, lt, a) and valid(L, ls, b):
                    col = c1(lt) if a == 1 else c2(lt)
                    out.append(X[b - 1][col])
                else:
                    out.append(mp.mpf(0))
        return out


def sommerfeld_mp(d, eps, lt, ls, a, b, n, m, rho, z, S, dps=30, path="auto") -> float:
    """S^n I^{ab}_nm by high-precision quadrature, any number of layers.

    ``path='real'`` integrates eq. scaledsommerfeldint along the real axis;
    ``path='contour'`` integrates eq. contourchange (K_m along the imaginary axis),
    the paper's form for rho > z; 'auto' picks the latter when rho > z.
    ``d=[]`` means sigma == 1.  Slow; for a handful of pins only."""
    import mpmath as mp
    if path == "auto":
        path = "contour" if rho > z else "real"
    with mp.workdps(dps):
        rho = mp.mpf(rho)
        z = mp.mpf(z)
        S = mp.mpf(S)
        norm = mp.sqrt(mp.factorial(n + m) * mp.factorial(n - m))

        def sig(k):
            if len(d) == 0:
                return mp.mpf(1)
            return sigma_mp(d, eps, lt, ls, k, dps)[2 * (a - 1) + (b - 1)]

        if path == "real":
            def f(k):
                return mp.besselj(m, k * rho) * (k * S) ** n * mp.exp(-k * z) * sig(k)
            kmax = (n + 1) / z + (dps + 10) * mp.log(10) / z + 4 * n / z
            step = min(mp.pi / rho if rho > 0 else kmax, 2 / z, kmax)
        else:
            j = mp.mpc(0, 1)
            sgn = (-1) ** (n + m)

            def f(t):
                br = mp.exp(-j * t * z) * sig(j * t) + sgn * mp.exp(j * t * z) * sig(-j * t)
                return mp.re(j ** (n - m) * mp.besselk(m, t * rho) * (S * t) ** n * br) / mp.pi
            kmax = (n + 1) / rho + (dps + 10) * mp.log(10) / rho + 4 * n / rho
            step = min(mp.pi / z, 2 / rho)
        pts = [mp.mpf(0)]
        while pts[-1] < kmax:
            pts.append(min(pts[-1] + step, kmax))
        val = mp.quad(f, pts)
        return float(val / norm)


# --------------------------------------------------------------------------
# octree keys
# --------------------------------------------------------------------------
def _spread21(v: np.ndarray) -> np.ndarray:
    """Bit i of a 21-bit integer goes to bit 3i (plain loop over bits)."""
    v = v.astype(np.uint64)
    out = np.zeros_like(v)
    for i in range(21):
        out |= ((v >> np.uint64(i)) & np.uint64(1)) << np.uint64(3 * i)
    return out


def morton_keys(x, y, h, x0, y0, scale) -> np.ndarray:
    """63-bit Morton key: 21-bit quantisation per axis, q = min(floor((c - c0) * scale),
    2^21 - 1) for x, y and the interface-relative height h (origin 0), interleaved
    with z in the top bit of each triple, then y, then x."""
    lim = np.float64(2 ** 21 - 1)

    def quant(c, c0):
        v = np.floor((np.asarray(c, np.float64) - np.float64(c0)) * np.float64(scale))
        return np.minimum(np.maximum(v, 0.0), lim).astype(np.uint64)
    qx, qy, qh = quant(x, x0), quant(y, y0), quant(h, 0.0)
    return (_spread21(qh) << np.uint64(2)) | (_spread21(qy) << np.uint64(1)) | _spread21(qx)


def morton_sort(keys: np.ndarray):
    """Stable sort by key (ties keep input order): returns (sorted keys, permutation)."""
    perm = np.argsort(keys, kind="stable")
    return keys[perm], perm.astype(np.int64)


def polarization_z(d, lt, ls, a, b, zs) -> float:
    """z-coordinate of the equivalent polarization source of eq. eqpolarizedsource
    for a source at height zs in layer ls and targets in layer lt."""
    if (a, b) == (1, 1):
        return d[lt] - (zs - d[ls])
    if (a, b) == (1, 2):
        return d[lt] - (d[ls - 1] - zs)
    if (a, b) == (2, 1):
        return d[lt - 1] + (zs - d[ls])
    return d[lt - 1] + (d[ls - 1] - zs)
