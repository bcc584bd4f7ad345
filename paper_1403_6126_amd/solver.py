"""Marshalling helper: holds the device tensors of one problem and calls the
C ABI.  No arithmetic of the method happens here; torch only allocates
device memory and provides the stream."""
from __future__ import annotations

import numpy as np

from . import rt


def quadrature_for(quad):
    """Angle table of a quadrature spec, from the library's own generator."""
    kind = quad[0]
    if kind == "gl":
        return rt.rt_quadrature(rt.RT_QUAD_GAUSS_LEGENDRE, int(quad[1]))
    if kind == "ls":
        return rt.rt_quadrature(rt.RT_QUAD_LEVEL_SYMMETRIC, int(quad[1]))
    if kind == "table":
        return np.asarray(quad[1], dtype=np.float64), np.asarray(quad[2], dtype=np.float64)
    raise ValueError(f"unknown quadrature {quad!r}")


class Solver:
    """One radiative-transfer problem resident on the GPU.

    ``wl`` is a workload description (grid, parameters, fields, initial
    intensity).  Intensities are angle-major ``(nang, ncell)``, as in the
    library; ``I0`` may be a numpy array or a device tensor (the latter
    avoids the host initialisation of large problems)."""

    def __init__(self, wl, precision: str | None = None, mu=None, w=None,
                 estimate_v: bool = True, I0=None, T0=None, newton_rtol=1e-14,
                 newton_maxit=64, device="cuda", feedback: bool = False,
                 original_transport: bool = False, c_reduced: float = 0.0,
                 second_order: bool = False):
        import torch
        self.torch = torch
        self.wl = wl
        prec = precision or wl.precision
        self.precision = rt.RT_FP32_MIXED if prec == "mixed" else rt.RT_FP64
        self.sdtype = torch.float32 if self.precision == rt.RT_FP32_MIXED else torch.float64
        if mu is None:
            mu, w = quadrature_for(wl.quad)
        self.mu = np.ascontiguousarray(mu, dtype=np.float64)
        self.w = np.ascontiguousarray(w, dtype=np.float64)
        self.nang = len(self.w)
        nc = wl.ncell
        self.ncell = nc
        grid = rt.make_grid(wl.ndim, wl.n, wl.dx, wl.bc)
        flags = (rt.RT_ESTIMATE_V if estimate_v else 0) | (rt.RT_GAS_FEEDBACK if feedback else 0) \
            | (rt.RT_ORIGINAL_TRANSPORT if original_transport else 0) \
            | (rt.RT_SECOND_ORDER if second_order else 0)
        params = rt.make_params(wl.C, wl.P, wl.gamma, wl.R, self.precision, flags, newton_rtol,
                                newton_maxit, c_reduced)
        self.ctx = rt.rt_create(grid, self.mu, self.w, params)
        dev = torch.device(device)
        f64 = dict(dtype=torch.float64, device=dev)

        def put(a):
            return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).to(dev)

        self.sa = put(wl.sigma_a)
        self.ss = put(wl.sigma_s)
        self.rho = put(wl.rho)
        self.T = put(wl.T if T0 is None else T0)
        self.v = put(wl.v).reshape(3, nc).contiguous()
        self.I = [torch.empty((self.nang, nc), dtype=self.sdtype, device=dev) for _ in range(2)]
        if I0 is None:
            I0 = wl.init(self.mu)
        if isinstance(I0, np.ndarray):
            I0 = torch.as_tensor(np.ascontiguousarray(I0, dtype=np.float64)).to(dev)
        self.I[0].copy_(I0)
        self.E = torch.zeros(nc, **f64)
        self.F = torch.zeros((3, nc), **f64)
        self.P = torch.zeros((6, nc), **f64)
        self.dEgas = torch.zeros(nc, **f64)
        self.dMom = torch.zeros((3, nc), **f64)
        self.totals = torch.zeros(rt.RT_NTOT, **f64)
        rt.rt_bind_intensity(self.ctx, self.I[0], self.I[1])
        if wl.ghost is not None:
            tables = wl.ghost(self.mu)
            for (axis, side), tab in tables.items():
                if axis < wl.ndim and wl.bc[axis][side] == rt.RT_BC_FIXED:
                    rt.rt_set_fixed_bc(self.ctx, axis, side, tab)
        if getattr(wl, "ghost_face", None) is not None:
            for (axis, side), tab in wl.ghost_face(self.mu).items():
                if axis < wl.ndim and wl.bc[axis][side] == rt.RT_BC_FIXED:
                    rt.rt_set_fixed_bc_face(self.ctx, axis, side, tab)
        self.fields = rt.make_fields(self.sa, self.ss, self.rho, self.T, self.v)
        self.out = rt.make_out(self.E, self.F, self.P, self.dEgas, self.dMom, self.totals)

    # ---------------------------------------------------------------- calls
    def _stream(self):
        return self.torch.cuda.current_stream().cuda_stream

    def step(self, nsteps: int = 1, dt: float | None = None):
        rt.rt_step(self.ctx, self.wl.dt if dt is None else dt, nsteps, self.fields, self.out,
                   self._stream())
        return self

    def moments(self):
        rt.rt_moments(self.ctx, self.out, self._stream())
        return self

    def transport(self, dt: float | None = None):
        """Transport increment as a device tensor (nang, ncell)."""
        dF = self.torch.empty_like(self.I[0])
        rt.rt_transport(self.ctx, self.wl.dt if dt is None else dt, self.fields, dF,
                        self._stream())
        return dF

    def source(self, dF, dt: float | None = None):
        rt.rt_source_implicit(self.ctx, self.wl.dt if dt is None else dt, self.fields, dF,
                              self.out, self._stream())
        return self

    def current(self):
        ptr = rt.rt_current_intensity(self.ctx)
        return self.I[0] if self.I[0].data_ptr() == ptr else self.I[1]

    def status(self) -> int:
        return rt.rt_sync_status(self.ctx)

    def state(self):
        """Host copies of the state and outputs (synchronises)."""
        self.torch.cuda.synchronize()
        return dict(I=self.current().double().cpu().numpy(), T=self.T.cpu().numpy(),
                    v=self.v.cpu().numpy(),
                    E=self.E.cpu().numpy(), F=self.F.cpu().numpy(), P=self.P.cpu().numpy(),
                    dEgas=self.dEgas.cpu().numpy(), dMom=self.dMom.cpu().numpy(),
                    totals=self.totals.cpu().numpy())

    def close(self):
        if getattr(self, "ctx", None):
            rt.rt_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
