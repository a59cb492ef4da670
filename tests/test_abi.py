"""C-ABI library checks that need no GPU: it loads, exports every function declared
in include/fmmlm.h, and rejects invalid arguments before touching the device."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "fmmlm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fmm\w+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    from paper_1908_10863_amd import fmmlm
    return fmmlm.lib()


def test_header_declares_the_plan_eval_pair():
    names = _declared()
    assert "fmm_layered_plan" in names and "fmm_layered_eval" in names


def test_library_exports_every_declared_symbol(L):
    for name in _declared():
        assert hasattr(L, name), name


def test_binding_covers_every_symbol():
    from paper_1908_10863_amd import fmmlm
    assert sorted(fmmlm.EXPORTS) == _declared()


def test_default_opts(L):
    from paper_1908_10863_amd import fmmlm
    o = fmmlm.Opts()
    L.fmmlm_default_opts(ctypes.byref(o))
    assert (o.leaf_cap, o.precision, o.fp64_top_levels, o.max_rhs, o.mac_d2) == (64, 0, 3, 1, 6)


def test_strerror_never_null(L):
    for code in range(-10, 1):
        s = L.fmm_layered_strerror(code)
        assert s is not None and len(s) > 0


def _plan_rc(L, d, eps, x, y, z, lay, p, opts=None):
    from paper_1908_10863_amd import fmmlm
    d = np.asarray(d, np.float64)
    eps = np.asarray(eps, np.float64)
    x, y, z = (np.asarray(a, np.float64) for a in (x, y, z))
    lay = np.asarray(lay, np.int32)
    h = ctypes.c_void_p()
    rc = L.fmm_layered_plan(len(d), ctypes.c_void_p(d.ctypes.data), ctypes.c_void_p(eps.ctypes.data),
                            len(x), ctypes.c_void_p(x.ctypes.data), ctypes.c_void_p(y.ctypes.data),
                            ctypes.c_void_p(z.ctypes.data), ctypes.c_void_p(lay.ctypes.data), p,
                            ctypes.byref(opts) if opts is not None else None, None, ctypes.byref(h))
    return rc, h


@pytest.mark.parametrize("case,code", [
    ("p0", -1), ("p17", -1), ("interfaces_up", -2), ("eps_neg", -3), ("eps_nan", -3),
    ("layer_range", -4), ("outside_layer", -4), ("nan_coord", -1), ("on_interface", -5),
    ("on_lower_interface", -5), ("near_interface", -5),
])
def test_plan_validation_errors(L, case, code):
    d, eps = [0.0, -1.0], [1.0, 5.0, 2.0]
    x, y, z, lay, p = [0.1, 0.2], [0.0, 0.1], [0.5, -0.5], [0, 1], 4
    if case == "p0":
        p = 0
    elif case == "p17":
        p = 17
    elif case == "interfaces_up":
        d = [-1.0, 0.0]
    elif case == "eps_neg":
        eps = [1.0, -5.0, 2.0]
    elif case == "eps_nan":
        eps = [1.0, float("nan"), 2.0]
    elif case == "layer_range":
        lay = [0, 3]
    elif case == "outside_layer":
        z = [0.5, 0.5]
    elif case == "nan_coord":
        x = [float("nan"), 0.2]
    elif case == "on_interface":
        z = [0.0, -0.5]            # layer 0's bottom interface d_0 = 0
    elif case == "on_lower_interface":
        z = [0.5, -1.0]            # layer 1's bottom interface d_1 = -1
    elif case == "near_interface":
        z = [1e-14, -0.5]          # below 1e-12 of the root box side above d_0
    rc, h = _plan_rc(L, d, eps, x, y, z, lay, p)
    assert rc == code
    assert not h.value


def test_reserved_options_rejected(L):
    from paper_1908_10863_amd import fmmlm
    o = fmmlm.Opts()
    L.fmmlm_default_opts(ctypes.byref(o))
    o.reserved[0] = 1
    rc, _ = _plan_rc(L, [0.0], [1.0, 2.0], [0.0], [0.0], [0.5], [0], 4, o)
    assert rc == -1


def test_mac_range_rejected(L):
    from paper_1908_10863_amd import fmmlm
    for bad in (3, 13):
        o = fmmlm.Opts()
        L.fmmlm_default_opts(ctypes.byref(o))
        o.mac_d2 = bad
        rc, _ = _plan_rc(L, [0.0], [1.0, 2.0], [0.0], [0.0], [0.5], [0], 4, o)
        assert rc == -1


def test_eval_rejects_null_plan(L):
    assert L.fmm_layered_eval(None, 1, None, 1, None, 1, 3, None) == -1


def test_plan_general_validates_coefficients(L):
    x, y, z, lay = (np.asarray(v, t) for v, t in (([0.1, 0.2], np.float64), ([0.0, 0.1], np.float64),
                                                   ([0.5, -0.5], np.float64), ([0, 1], np.int32)))
    d = np.array([0.0, -1.0])

    def rc_of(a, b):
        a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
        h = ctypes.c_void_p()
        return L.fmm_layered_plan_general(2, ctypes.c_void_p(d.ctypes.data), ctypes.c_void_p(a.ctypes.data),
                                          ctypes.c_void_p(b.ctypes.data), 2, ctypes.c_void_p(x.ctypes.data),
                                          ctypes.c_void_p(y.ctypes.data), ctypes.c_void_p(z.ctypes.data),
                                          ctypes.c_void_p(lay.ctypes.data), 4, None, None, ctypes.byref(h)), h

    for a, b in (([1.0, -1.0, 1.0], [1.0, 2.0, 3.0]), ([1.0, 1.0, 1.0], [1.0, 0.0, 3.0]),
                 ([1.0, float("nan"), 1.0], [1.0, 2.0, 3.0]), ([1.0, 1.0, 1.0], [float("inf"), 2.0, 3.0])):
        rc, h = rc_of(a, b)
        assert rc == -3 and not h.value
    h = ctypes.c_void_p()
    assert L.fmm_layered_plan_general(2, None, None, None, 2, None, None, None, None, 4, None, None,
                                      ctypes.byref(h)) == -1


def test_solve_rejects_null_plan(L):
    from paper_1908_10863_amd import fmmlm
    info = fmmlm.SolveInfo()
    assert L.fmm_layered_solve(None, None, None, None, None, None, ctypes.byref(info)) == -1


def test_python_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_1908_10863_amd import fmmlm
    monkeypatch.setattr(fmmlm, "_lib", None)
    monkeypatch.setattr(fmmlm, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError):
        fmmlm.lib()


_CTYPE = {"int32_t": ctypes.c_int32, "int64_t": ctypes.c_int64, "uint64_t": ctypes.c_uint64,
          "double": ctypes.c_double, "float": ctypes.c_float, "fmmlm_surrogate_t": ctypes.c_void_p}


def _header_struct(name):
    """(field, ctypes type) of `typedef struct {...} name;` in include/fmmlm.h, in order."""
    src = open(os.path.join(ROOT, "include", "fmmlm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    body = re.search(r"typedef struct \{([^{}]*)\}\s*" + name + r"\s*;", src).group(1)
    out = []
    for ty, names in re.findall(r"(\w+)\s+([^;]+);", body):  # "type a, b[3];"
        t = _CTYPE[ty]
        for fld, n in re.findall(r"(\w+)\s*(?:\[(\d+)\])?", names):
            out.append((fld, t * int(n) if n else t))
    return out


@pytest.mark.parametrize("cname,pyname", [("fmmlm_opts", "Opts"), ("fmmlm_stats", "Stats"),
                                          ("fmmlm_solve_opts", "SolveOpts"), ("fmmlm_solve_info", "SolveInfo"),
                                          ("fmmlm_train_opts", "TrainOpts"),
                                          ("fmmlm_train_report", "TrainReport")])
def test_binding_structs_match_the_header(cname, pyname):
    """Every struct the binding passes across the boundary has the header's fields, in the
    header's order and with its types, so offsets and size agree with the C layout."""
    from paper_1908_10863_amd import fmmlm
    hdr = _header_struct(cname)
    py = getattr(fmmlm, pyname)._fields_
    assert [f for f, _ in py] == [f for f, _ in hdr], cname
    for (f, tp), (_, th) in zip(py, hdr):
        assert ctypes.sizeof(tp) == ctypes.sizeof(th) and getattr(tp, "_type_", tp) == getattr(th, "_type_", th), (cname, f)
