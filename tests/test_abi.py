"""Host-side checks of the C ABI (no GPU work): every symbol declared in
include/*.h is exported, the library's quadrature equals the oracle's,
argument validation rejects bad input before touching the device, and the
product package never reaches the oracle."""
import ctypes as ct
import os
import re
import subprocess

import numpy as np
import pytest

from paper_1403_6126_amd import rt

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if h.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", h)).read()
            names |= set(re.findall(r"^\s*(?:int|double|const char \*)\s*(rt_\w+)\s*\(",
                                    txt, re.M))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    names = _declared()
    assert len(names) >= 15
    L = ct.CDLL(rt.LIB_PATH)
    for n in names:
        assert hasattr(L, n), n
    bound = {s[0] for s in rt.SIGNATURES}
    assert set(names) == bound


def test_quadrature_matches_oracle():
    from oracle.quadrature import gauss_legendre, level_symmetric
    for order in (2, 4, 6, 8, 10, 12):
        mu, w = rt.rt_quadrature(rt.RT_QUAD_LEVEL_SYMMETRIC, order)
        mo, wo = level_symmetric(order)
        assert np.array_equal(mu, mo) or np.abs(mu - mo).max() <= 1e-15
        assert np.abs(w - wo).max() <= 2e-15
    for order in (14, 16):
        mu, w = rt.rt_quadrature(rt.RT_QUAD_LEVEL_SYMMETRIC, order)
        mo, wo = level_symmetric(order)
        assert np.abs(mu - mo).max() <= 1e-15
        assert np.abs(w - wo).max() <= 1e-12
        assert abs(w.sum() - 1) <= 1e-14
        assert np.abs(np.einsum("m,mi,mj->ij", w, mu, mu) - np.eye(3) / 3).max() <= 1e-14
    for n in (2, 16, 64, 288):
        mu, w = rt.rt_quadrature(rt.RT_QUAD_GAUSS_LEGENDRE, n)
        mo, wo = gauss_legendre(n)
        assert np.abs(mu - mo).max() <= 1e-15 and np.abs(w - wo).max() <= 1e-15


def test_quadrature_rejects_bad_orders():
    for kind, order in [(rt.RT_QUAD_LEVEL_SYMMETRIC, 3), (rt.RT_QUAD_LEVEL_SYMMETRIC, 18),
                        (rt.RT_QUAD_GAUSS_LEGENDRE, 5), (7, 4)]:
        assert rt.lib().rt_quadrature(kind, order, None, None, 0) == rt.RT_EINVAL


def _grid():
    return rt.make_grid(3, (4, 4, 4), (0.25, 0.25, 0.25), ((0, 0),) * 3)


@pytest.mark.parametrize("case", ["weights", "norm", "ndim", "bc", "c", "gamma", "cells",
                                  "angles", "c_reduced_above_c", "c_reduced_negative",
                                  "c_reduced_with_estimate"])
def test_create_validation_before_device(case):
    mu, w = rt.rt_quadrature(rt.RT_QUAD_LEVEL_SYMMETRIC, 4)
    g = _grid()
    p = rt.make_params(1.0, 1.0, 5 / 3, 1.0)
    expect = rt.RT_EINVAL
    if case == "weights":
        w = w * 1.01
        expect = rt.RT_EBADQUAD
    elif case == "norm":
        mu = mu * 1.001
        expect = rt.RT_EBADQUAD
    elif case == "ndim":
        g.ndim = 2                       # n[2] = 4 on an unused axis
    elif case == "bc":
        g.bc[0][0] = rt.RT_BC_FIXED      # periodic on one side only
    elif case == "c":
        p.c = 0.0
    elif case == "gamma":
        p.gamma = 1.0
    elif case == "cells":                # cell indices are 32-bit
        g = rt.make_grid(3, (2048, 2048, 1024), (1.0, 1.0, 1.0), ((0, 0),) * 3)
        expect = rt.RT_EUNSUPPORTED
    elif case == "angles":               # more than RT_MAX_ANGLES directions
        n = 1026
        phi = np.arange(n) * 2 * np.pi / n
        mu = np.stack([np.cos(phi), np.sin(phi), np.zeros(n)], axis=1)
        w = np.full(n, 1.0 / n)
    elif case == "c_reduced_above_c":
        p = rt.make_params(1.0, 1.0, 5 / 3, 1.0, flags=0, c_reduced=1.5)
    elif case == "c_reduced_negative":
        p = rt.make_params(1.0, 1.0, 5 / 3, 1.0, flags=0, c_reduced=-0.5)
    elif case == "c_reduced_with_estimate":
        p = rt.make_params(1.0, 1.0, 5 / 3, 1.0, flags=rt.RT_ESTIMATE_V, c_reduced=0.5)
        expect = rt.RT_EUNSUPPORTED
    with pytest.raises(rt.RTError) as ei:
        rt.rt_create(g, mu, w, p)
    assert ei.value.status == expect


def test_product_package_does_not_use_oracle():
    pkg = os.path.join(ROOT, "paper_1403_6126_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".cpp", ".h", ".inc")):
                txt = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(import|from)\s+oracle", txt, re.M), f
                assert "rt_oracle" not in txt, f
    out = subprocess.run(["ldd", rt.LIB_PATH], capture_output=True, text=True).stdout
    assert "oracle" not in out


@pytest.mark.parametrize("field,value", [("pool_bytes", 0), ("max_active", 0),
                                         ("chunk_work", 0), ("large_work", 0),
                                         ("packed_cells", -1)])
def test_serve_config_validation_before_device(field, value):
    cfg = dict(pool_bytes=1 << 30, max_active=4, packed_cells=0, chunk_work=1, large_work=1)
    cfg[field] = value
    with pytest.raises(rt.RTError) as ei:
        rt.rt_serve_create(**cfg)
    assert ei.value.status == rt.RT_EINVAL


def test_headers_are_plain_c(tmp_path):
    """The boundary headers compile as strict C99 (plain pointers and sizes,
    no C++ or torch types), and every declared function is callable from C."""
    src = tmp_path / "use.c"
    src.write_text('#include "rt.h"\n#include "rt_serve.h"\n'
                   "int use(void) {\n"
                   "  rt_params p; rt_request r; rt_serve_config s;\n"
                   "  (void)p; (void)r; (void)s;\n"
                   "  return (int)sizeof(rt_fields) + (int)sizeof(rt_out);\n"
                   "}\n")
    r = subprocess.run(["gcc", "-std=c99", "-pedantic", "-Wall", "-Wextra", "-Werror",
                        "-I", os.path.join(ROOT, "include"), "-c", str(src), "-o",
                        str(tmp_path / "use.o")], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
