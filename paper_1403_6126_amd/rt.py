"""ctypes binding of the C ABI in ``include/rt.h`` and ``include/rt_serve.h``
(argument marshalling only).

Every function here has the name of the C entry point it calls.  Device
arrays are passed as raw pointers (``int``), e.g. ``tensor.data_ptr()`` of a
torch tensor; streams as the integer handle of a ``hipStream_t`` (torch:
``torch.cuda.current_stream().cuda_stream``).  Errors become ``RTError``.
The library must have been built (``paper_1403_6126_amd.build.build()``):
there is no fallback implementation.
"""
from __future__ import annotations

import ctypes as ct
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librt.so")

RT_PENDING = 1
RT_OK, RT_EINVAL, RT_ENOMEM, RT_EDEVICE, RT_ECFL, RT_ENOCONV, RT_EBADQUAD, RT_ESTATE, \
    RT_EUNSUPPORTED, RT_ETOOBIG = 0, -1, -2, -3, -4, -5, -6, -7, -8, -9
RT_STATIC_SCRATCH_BYTES = 64 << 20
RT_BC_PERIODIC, RT_BC_FIXED, RT_BC_COPY, RT_BC_VACUUM = 0, 1, 2, 3
RT_FP64, RT_FP32_MIXED = 0, 1
RT_QUAD_GAUSS_LEGENDRE, RT_QUAD_LEVEL_SYMMETRIC = 0, 1
RT_ESTIMATE_V = 1
RT_GAS_FEEDBACK = 2
RT_ORIGINAL_TRANSPORT = 4
RT_SECOND_ORDER = 8
RT_NTOT = 12
RT_MAX_ANGLES = 1024


class RTError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {rt_strerror(status)} ({status})")


class rt_grid(ct.Structure):
    _fields_ = [("ndim", ct.c_int), ("n", ct.c_int * 3), ("dx", ct.c_double * 3),
                ("bc", (ct.c_int * 2) * 3)]


class rt_angles(ct.Structure):
    _fields_ = [("n", ct.c_int), ("mu", ct.POINTER(ct.c_double)),
                ("w", ct.POINTER(ct.c_double))]


class rt_params(ct.Structure):
    _fields_ = [("c", ct.c_double), ("prat", ct.c_double), ("gamma", ct.c_double),
                ("r_ideal", ct.c_double), ("precision", ct.c_int), ("flags", ct.c_uint),
                ("newton_rtol", ct.c_double), ("newton_maxit", ct.c_int),
                ("c_reduced", ct.c_double)]


class rt_fields(ct.Structure):
    _fields_ = [("sigma_a", ct.c_void_p), ("sigma_s", ct.c_void_p), ("rho", ct.c_void_p),
                ("T", ct.c_void_p), ("v", ct.c_void_p)]


class rt_out(ct.Structure):
    _fields_ = [("Er", ct.c_void_p), ("Fr", ct.c_void_p), ("Pr", ct.c_void_p),
                ("dEgas", ct.c_void_p), ("dMom", ct.c_void_p), ("totals", ct.c_void_p)]


class rt_info(ct.Structure):
    _fields_ = [("nang", ct.c_int), ("ncell", ct.c_longlong), ("storage_bytes", ct.c_int),
                ("block_threads", ct.c_int), ("grid_blocks", ct.c_longlong)]


class rt_serve_config(ct.Structure):
    _fields_ = [("pool_bytes", ct.c_ulonglong), ("max_active", ct.c_int),
                ("packed_cells", ct.c_longlong), ("chunk_work", ct.c_longlong),
                ("large_work", ct.c_longlong)]


class rt_request(ct.Structure):
    _fields_ = [("grid", rt_grid), ("angles", rt_angles), ("params", rt_params),
                ("dt", ct.c_double), ("nsteps", ct.c_int), ("ghost", ct.c_void_p),
                ("sigma_a", ct.c_void_p), ("sigma_s", ct.c_void_p), ("rho", ct.c_void_p),
                ("T", ct.c_void_p), ("v", ct.c_void_p), ("I0", ct.c_void_p),
                ("T_out", ct.c_void_p), ("Er", ct.c_void_p), ("Fr", ct.c_void_p),
                ("totals", ct.c_void_p), ("I_out", ct.c_void_p)]


class rt_serve_result(ct.Structure):
    _fields_ = [("status", ct.c_int), ("packed", ct.c_int), ("t_submit", ct.c_double),
                ("t_admit", ct.c_double), ("t_done", ct.c_double)]


class rt_serve_counters(ct.Structure):
    _fields_ = [("submitted", ct.c_longlong), ("completed", ct.c_longlong),
                ("active", ct.c_longlong), ("peak_active", ct.c_longlong),
                ("pool_bytes", ct.c_ulonglong), ("pool_used", ct.c_ulonglong),
                ("peak_pool_used", ct.c_ulonglong), ("packed_launches", ct.c_longlong),
                ("packed_requests", ct.c_longlong), ("chunk_launches", ct.c_longlong),
                ("cell_angle_updates", ct.c_double)]


_lib = None

# (name, restype, argtypes) of every exported entry point of include/rt.h
SIGNATURES = [
    ("rt_quadrature", ct.c_int, [ct.c_int, ct.c_int, ct.POINTER(ct.c_double),
                                 ct.POINTER(ct.c_double), ct.c_int]),
    ("rt_create", ct.c_int, [ct.POINTER(rt_grid), ct.POINTER(rt_angles), ct.POINTER(rt_params),
                             ct.POINTER(ct.c_void_p)]),
    ("rt_destroy", ct.c_int, [ct.c_void_p]),
    ("rt_bind_intensity", ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_void_p]),
    ("rt_current_intensity", ct.c_int, [ct.c_void_p, ct.POINTER(ct.c_void_p)]),
    ("rt_set_fixed_bc", ct.c_int, [ct.c_void_p, ct.c_int, ct.c_int, ct.POINTER(ct.c_double)]),
    ("rt_set_fixed_bc_face", ct.c_int, [ct.c_void_p, ct.c_int, ct.c_int,
                                        ct.POINTER(ct.c_double)]),
    ("rt_moments", ct.c_int, [ct.c_void_p, ct.POINTER(rt_out), ct.c_void_p]),
    ("rt_transport", ct.c_int, [ct.c_void_p, ct.c_double, ct.POINTER(rt_fields), ct.c_void_p,
                                ct.c_void_p]),
    ("rt_source_implicit", ct.c_int, [ct.c_void_p, ct.c_double, ct.POINTER(rt_fields),
                                      ct.c_void_p, ct.POINTER(rt_out), ct.c_void_p]),
    ("rt_step", ct.c_int, [ct.c_void_p, ct.c_double, ct.c_int, ct.POINTER(rt_fields),
                           ct.POINTER(rt_out), ct.c_void_p]),
    ("rt_step_static", ct.c_int, [ct.POINTER(rt_grid), ct.POINTER(rt_angles),
                                  ct.POINTER(rt_params), ct.c_void_p, ct.c_void_p, ct.c_double,
                                  ct.c_int, ct.POINTER(rt_fields), ct.POINTER(rt_out),
                                  ct.c_void_p, ct.c_void_p]),
    ("rt_equilibrium_intensity", ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_void_p,
                                            ct.c_void_p]),
    ("rt_sync_status", ct.c_int, [ct.c_void_p]),
    ("rt_profile_enable", ct.c_int, [ct.c_void_p, ct.c_int]),
    ("rt_profile_read", ct.c_int, [ct.c_void_p, ct.POINTER(ct.c_double), ct.POINTER(ct.c_int)]),
    ("rt_get_info", ct.c_int, [ct.c_void_p, ct.POINTER(rt_info)]),
    ("rt_strerror", ct.c_char_p, [ct.c_int]),
    # include/rt_serve.h
    ("rt_serve_create", ct.c_int, [ct.POINTER(rt_serve_config), ct.POINTER(ct.c_void_p)]),
    ("rt_serve_submit", ct.c_int, [ct.c_void_p, ct.POINTER(rt_request),
                                   ct.POINTER(ct.c_longlong)]),
    ("rt_serve_poll", ct.c_int, [ct.c_void_p, ct.c_longlong, ct.POINTER(rt_serve_result)]),
    ("rt_serve_wait", ct.c_int, [ct.c_void_p, ct.c_longlong, ct.POINTER(rt_serve_result)]),
    ("rt_serve_now", ct.c_double, [ct.c_void_p]),
    ("rt_serve_get_counters", ct.c_int, [ct.c_void_p, ct.POINTER(rt_serve_counters)]),
    ("rt_serve_destroy", ct.c_int, [ct.c_void_p]),
]


def lib():
    """The loaded HIP library; raises if it has not been built.

    torch is imported first: its ROCm build carries its own HIP runtime,
    which the library then binds to (same soname), so that the process holds
    one HIP runtime and torch's streams and allocations are valid handles
    for the library.  Loading the library first would bring in the system
    runtime, and torch would then load a second one."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library {LIB_PATH} is not built; run "
                               "paper_1403_6126_amd.build.build() first (no fallback exists)")
        try:
            import torch  # noqa: F401  (one HIP runtime per process, see above)
        except ImportError:
            pass
        L = ct.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(st: int, where: str) -> int:
    if st < 0:
        raise RTError(st, where)
    return st


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ct.POINTER(ct.c_double))


def _vp(x):
    if x is None:
        return None
    if hasattr(x, "data_ptr"):
        return ct.c_void_p(x.data_ptr())
    return ct.c_void_p(int(x))


# ------------------------------------------------------------ entry points
def rt_strerror(status: int) -> str:
    return lib().rt_strerror(status).decode()


def rt_quadrature(kind: int, order: int):
    n = _check(lib().rt_quadrature(kind, order, None, None, 0), "rt_quadrature")
    mu = np.zeros((n, 3))
    w = np.zeros(n)
    _check(lib().rt_quadrature(kind, order, _dptr(mu), _dptr(w), n), "rt_quadrature")
    return mu, w


def make_grid(ndim, n, dx, bc) -> rt_grid:
    g = rt_grid()
    g.ndim = ndim
    for d in range(3):
        g.n[d] = int(n[d])
        g.dx[d] = float(dx[d])
        for s in range(2):
            g.bc[d][s] = int(bc[d][s])
    return g


def make_params(c, prat, gamma, r_ideal, precision=RT_FP64, flags=RT_ESTIMATE_V,
                newton_rtol=1e-14, newton_maxit=64, c_reduced=0.0) -> rt_params:
    return rt_params(c, prat, gamma, r_ideal, precision, flags, newton_rtol, newton_maxit,
                     c_reduced)


def rt_create(grid: rt_grid, mu: np.ndarray, w: np.ndarray, params: rt_params) -> int:
    mu = np.ascontiguousarray(mu, dtype=np.float64)
    w = np.ascontiguousarray(w, dtype=np.float64)
    ang = rt_angles(len(w), _dptr(mu), _dptr(w))
    out = ct.c_void_p()
    _check(lib().rt_create(ct.byref(grid), ct.byref(ang), ct.byref(params), ct.byref(out)),
           "rt_create")
    return out.value


def rt_destroy(ctx: int) -> None:
    _check(lib().rt_destroy(ct.c_void_p(ctx)), "rt_destroy")


def rt_bind_intensity(ctx: int, I_a, I_b) -> None:
    _check(lib().rt_bind_intensity(ct.c_void_p(ctx), _vp(I_a), _vp(I_b)), "rt_bind_intensity")


def rt_current_intensity(ctx: int) -> int:
    out = ct.c_void_p()
    _check(lib().rt_current_intensity(ct.c_void_p(ctx), ct.byref(out)), "rt_current_intensity")
    return out.value


def rt_set_fixed_bc(ctx: int, axis: int, side: int, table: np.ndarray) -> None:
    t = np.ascontiguousarray(table, dtype=np.float64)
    _check(lib().rt_set_fixed_bc(ct.c_void_p(ctx), axis, side, _dptr(t)), "rt_set_fixed_bc")


def rt_set_fixed_bc_face(ctx: int, axis: int, side: int, table: np.ndarray) -> None:
    """table: (nang, ncell // n[axis]) ghost intensities of the face cells."""
    t = np.ascontiguousarray(table, dtype=np.float64)
    _check(lib().rt_set_fixed_bc_face(ct.c_void_p(ctx), axis, side, _dptr(t)),
           "rt_set_fixed_bc_face")


def make_fields(sigma_a, sigma_s, rho, T, v) -> rt_fields:
    return rt_fields(_vp(sigma_a), _vp(sigma_s), _vp(rho), _vp(T), _vp(v))


def make_out(Er=None, Fr=None, Pr=None, dEgas=None, dMom=None, totals=None) -> rt_out:
    return rt_out(_vp(Er), _vp(Fr), _vp(Pr), _vp(dEgas), _vp(dMom), _vp(totals))


def rt_moments(ctx: int, out: rt_out | None, stream=0) -> None:
    _check(lib().rt_moments(ct.c_void_p(ctx), ct.byref(out) if out is not None else None,
                            ct.c_void_p(stream)), "rt_moments")


def rt_transport(ctx: int, dt: float, fields: rt_fields, dF, stream=0) -> None:
    _check(lib().rt_transport(ct.c_void_p(ctx), dt, ct.byref(fields), _vp(dF),
                              ct.c_void_p(stream)), "rt_transport")


def rt_source_implicit(ctx: int, dt: float, fields: rt_fields, dF, out: rt_out | None,
                       stream=0) -> None:
    _check(lib().rt_source_implicit(ct.c_void_p(ctx), dt, ct.byref(fields), _vp(dF),
                                    ct.byref(out) if out is not None else None,
                                    ct.c_void_p(stream)), "rt_source_implicit")


def rt_step(ctx: int, dt: float, nsteps: int, fields: rt_fields, out: rt_out | None,
            stream=0) -> None:
    _check(lib().rt_step(ct.c_void_p(ctx), dt, nsteps, ct.byref(fields),
                         ct.byref(out) if out is not None else None, ct.c_void_p(stream)),
           "rt_step")


def rt_step_static(grid: rt_grid, mu: np.ndarray, w: np.ndarray, params: rt_params, I_a, I_b,
                   dt: float, nsteps: int, fields: rt_fields, out: rt_out | None, status,
                   stream=0) -> None:
    mu = np.ascontiguousarray(mu, dtype=np.float64)
    w = np.ascontiguousarray(w, dtype=np.float64)
    ang = rt_angles(len(w), _dptr(mu), _dptr(w))
    _check(lib().rt_step_static(ct.byref(grid), ct.byref(ang), ct.byref(params), _vp(I_a),
                                _vp(I_b), dt, nsteps, ct.byref(fields),
                                ct.byref(out) if out is not None else None, _vp(status),
                                ct.c_void_p(stream)), "rt_step_static")


def rt_equilibrium_intensity(ctx: int, T, I, stream=0) -> None:
    _check(lib().rt_equilibrium_intensity(ct.c_void_p(ctx), _vp(T), _vp(I), ct.c_void_p(stream)),
           "rt_equilibrium_intensity")


def rt_sync_status(ctx: int) -> int:
    return lib().rt_sync_status(ct.c_void_p(ctx))


def rt_profile_enable(ctx: int, enable: bool) -> None:
    _check(lib().rt_profile_enable(ct.c_void_p(ctx), 1 if enable else 0), "rt_profile_enable")


def rt_profile_read(ctx: int):
    ms = ct.c_double()
    n = ct.c_int()
    _check(lib().rt_profile_read(ct.c_void_p(ctx), ct.byref(ms), ct.byref(n)), "rt_profile_read")
    return ms.value, n.value


def rt_get_info(ctx: int) -> rt_info:
    info = rt_info()
    _check(lib().rt_get_info(ct.c_void_p(ctx), ct.byref(info)), "rt_get_info")
    return info


# ----------------------------------------------------------------- serving
def rt_serve_create(pool_bytes: int, max_active: int, packed_cells: int, chunk_work: int,
                    large_work: int) -> int:
    cfg = rt_serve_config(pool_bytes, max_active, packed_cells, chunk_work, large_work)
    out = ct.c_void_p()
    _check(lib().rt_serve_create(ct.byref(cfg), ct.byref(out)), "rt_serve_create")
    return out.value


def rt_serve_submit(srv: int, req: rt_request) -> int:
    rid = ct.c_longlong()
    _check(lib().rt_serve_submit(ct.c_void_p(srv), ct.byref(req), ct.byref(rid)),
           "rt_serve_submit")
    return rid.value


def rt_serve_poll(srv: int, rid: int):
    """None while the request is in flight, else its rt_serve_result."""
    res = rt_serve_result()
    st = _check(lib().rt_serve_poll(ct.c_void_p(srv), rid, ct.byref(res)), "rt_serve_poll")
    return None if st == RT_PENDING else res


def rt_serve_wait(srv: int, rid: int) -> rt_serve_result:
    res = rt_serve_result()
    _check(lib().rt_serve_wait(ct.c_void_p(srv), rid, ct.byref(res)), "rt_serve_wait")
    return res


def rt_serve_now(srv: int) -> float:
    return lib().rt_serve_now(ct.c_void_p(srv))


def rt_serve_get_counters(srv: int) -> rt_serve_counters:
    c = rt_serve_counters()
    _check(lib().rt_serve_get_counters(ct.c_void_p(srv), ct.byref(c)), "rt_serve_get_counters")
    return c


def rt_serve_destroy(srv: int) -> None:
    _check(lib().rt_serve_destroy(ct.c_void_p(srv)), "rt_serve_destroy")
