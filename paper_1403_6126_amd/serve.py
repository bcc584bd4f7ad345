"""Client side of the serving runtime (``include/rt_serve.h``).

Marshals workloads into requests of the C server, replays arrival traces
against it, and runs the same traces through the plain path (one
``rt_create`` / ``rt_step`` at a time, first come first served) for
comparison.  No arithmetic of the method happens here.
"""
from __future__ import annotations

import threading
import time
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence

import numpy as np

from . import rt
from .solver import quadrature_for


@dataclass
class Handle:
    """A submitted request and the host arrays it reads and writes."""
    rid: int
    wl: object
    nang: int
    work: float
    arrays: Dict[str, np.ndarray] = field(default_factory=dict)
    result: Optional[Dict] = None


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


class Server:
    """One serving runtime on the current GPU (see ``include/rt_serve.h``)."""

    def __init__(self, pool_bytes: int = 32 << 30, max_active: int = 1024,
                 packed_cells: int = 512, chunk_work: int = 200_000_000,
                 large_work: int = 20_000_000):
        self.srv = rt.rt_serve_create(int(pool_bytes), int(max_active), int(packed_cells),
                                      int(chunk_work), int(large_work))
        self._lock = threading.Lock()

    def submit(self, wl, mu=None, w=None, I0: Optional[np.ndarray] = None,
               keep_I: bool = False) -> Handle:
        if mu is None:
            mu, w = quadrature_for(wl.quad)
        mu, w = _f64(mu), _f64(w)
        nang, nc = len(w), wl.ncell
        prec = rt.RT_FP32_MIXED if wl.precision == "mixed" else rt.RT_FP64
        sdt = np.float32 if prec == rt.RT_FP32_MIXED else np.float64
        a = dict(mu=mu, w=w, sa=_f64(wl.sigma_a), ss=_f64(wl.sigma_s), rho=_f64(wl.rho),
                 T=_f64(wl.T), v=_f64(np.reshape(wl.v, (3, nc))),
                 T_out=np.empty(nc), E=np.empty(nc), F=np.empty((3, nc)),
                 totals=np.empty(rt.RT_NTOT))
        if I0 is not None:
            a["I0"] = np.ascontiguousarray(I0, dtype=sdt)
        if keep_I:
            a["I"] = np.empty((nang, nc), dtype=sdt)
        if wl.ghost is not None:
            g = np.zeros((3, 2, nang))
            for (axis, side), tab in wl.ghost(mu).items():
                g[axis, side] = tab
            a["ghost"] = g
        req = rt.rt_request()
        req.grid = rt.make_grid(wl.ndim, wl.n, wl.dx, wl.bc)
        req.angles = rt.rt_angles(nang, rt._dptr(mu), rt._dptr(w))
        req.params = rt.make_params(wl.C, wl.P, wl.gamma, wl.R, prec)
        req.dt = wl.dt
        req.nsteps = int(wl.nsteps)
        req.ghost = _ptr(a.get("ghost"))
        req.sigma_a, req.sigma_s, req.rho = _ptr(a["sa"]), _ptr(a["ss"]), _ptr(a["rho"])
        req.T, req.v = _ptr(a["T"]), _ptr(a["v"])
        req.I0 = _ptr(a.get("I0"))
        req.T_out, req.Er, req.Fr = _ptr(a["T_out"]), _ptr(a["E"]), _ptr(a["F"])
        req.totals, req.I_out = _ptr(a["totals"]), _ptr(a.get("I"))
        rid = rt.rt_serve_submit(self.srv, req)
        return Handle(rid, wl, nang, float(nc) * nang * wl.nsteps, a)

    def _result(self, h: Handle, res) -> Dict:
        a = h.arrays
        h.result = dict(status=res.status, packed=bool(res.packed), t_submit=res.t_submit,
                        t_admit=res.t_admit, t_done=res.t_done, T=a["T_out"], E=a["E"],
                        F=a["F"], totals=a["totals"], I=a.get("I"))
        return h.result

    def wait(self, h: Handle) -> Dict:
        return self._result(h, rt.rt_serve_wait(self.srv, h.rid))

    def poll(self, h: Handle) -> Optional[Dict]:
        res = rt.rt_serve_poll(self.srv, h.rid)
        return None if res is None else self._result(h, res)

    def now(self) -> float:
        return rt.rt_serve_now(self.srv)

    def counters(self) -> Dict:
        c = rt.rt_serve_get_counters(self.srv)
        return {k: getattr(c, k) for k, _ in c._fields_}

    def close(self):
        if getattr(self, "srv", None):
            rt.rt_serve_destroy(self.srv)
            self.srv = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _percentiles(lat: Sequence[float]) -> Dict[str, float]:
    x = np.sort(np.asarray(lat, dtype=np.float64))
    return dict(p50=float(np.percentile(x, 50)), p99=float(np.percentile(x, 99)),
                mean=float(x.mean()), max=float(x.max()))


def request_class(wl, nang: int, packed_cells: int, large_work: int) -> str:
    """The server's class of a request: 'packed' (FP32-mixed, at most
    packed_cells cells: one workgroup per solve), 'large' (at least
    large_work updates per step: the large-request stream), else 'chunked'."""
    if wl.precision == "mixed" and wl.ncell <= packed_cells:
        return "packed"
    return "large" if wl.ncell * nang >= large_work else "chunked"


def _by_class(lat: Sequence[float], classes: Sequence[str]) -> Dict[str, Dict]:
    out = {}
    for c in ("packed", "chunked", "large"):
        x = [l for l, k in zip(lat, classes) if k == c]
        if x:
            out[c] = dict(count=len(x), **_percentiles(x))
    return out


def run_batched(wls: List, arrivals: Sequence[float], progress=None, **server_kw) -> Dict:
    """Replays the trace against the server: request i is submitted at
    arrivals[i] seconds after the start; returns latencies (submission to
    results in host memory) and aggregate throughput."""
    with Server(**server_kw) as s:
        handles: List[Optional[Handle]] = [None] * len(wls)
        t0 = s.now()
        for i, wl in enumerate(wls):
            delay = t0 + arrivals[i] - s.now()
            if delay > 0:
                time.sleep(delay)
            handles[i] = s.submit(wl)
            if progress and (i + 1) % 50 == 0:
                progress(f"submitted {i + 1}/{len(wls)}")
        res = []
        for i, h in enumerate(handles):
            res.append(s.wait(h))
            if progress and (i + 1) % 50 == 0:
                progress(f"completed {i + 1}/{len(wls)}")
        counters = s.counters()
    bad = [r["status"] for r in res if r["status"] != rt.RT_OK]
    if bad:
        raise RuntimeError(f"{len(bad)} served requests failed (first status {bad[0]})")
    lat = [r["t_done"] - r["t_submit"] for r in res]
    first = min(r["t_submit"] for r in res)
    last = max(r["t_done"] for r in res)
    work = sum(h.work for h in handles)
    out = dict(requests=len(wls), makespan_s=last - first, updates=work,
               throughput=work / (last - first), packed=sum(r["packed"] for r in res),
               peak_active=counters["peak_active"],
               peak_pool_gb=counters["peak_pool_used"] / 1e9,
               chunk_launches=counters["chunk_launches"],
               packed_launches=counters["packed_launches"])
    out.update({f"latency_{k}_s": v for k, v in _percentiles(lat).items()})
    classes = [request_class(h.wl, h.nang, server_kw.get("packed_cells", 4096),
                             server_kw.get("large_work", 20_000_000)) for h in handles]
    out["latency_by_class_s"] = _by_class(lat, classes)
    return out


def run_fifo(wls: List, arrivals: Sequence[float], progress=None, packed_cells: int = 512,
             large_work: int = 20_000_000) -> Dict:
    """The same trace through the plain path: one request at a time in
    arrival order, each created, uploaded, stepped with rt_step, copied back
    and destroyed before the next starts.  Latencies are also grouped by the
    class the server would give each request."""
    import torch
    dev = torch.device("cuda")
    stream = torch.cuda.current_stream().cuda_stream
    lat, classes, t_first, t_last, work = [], [], None, 0.0, 0.0
    t0 = time.perf_counter()
    for i, wl in enumerate(wls):
        arrive = t0 + arrivals[i]
        now = time.perf_counter()
        if now < arrive:
            time.sleep(arrive - now)
        mu, w = quadrature_for(wl.quad)
        nang, nc = len(w), wl.ncell
        prec = rt.RT_FP32_MIXED if wl.precision == "mixed" else rt.RT_FP64
        sdt = torch.float32 if prec == rt.RT_FP32_MIXED else torch.float64
        ctx = rt.rt_create(rt.make_grid(wl.ndim, wl.n, wl.dx, wl.bc), mu, w,
                           rt.make_params(wl.C, wl.P, wl.gamma, wl.R, prec))
        try:
            put = lambda x: torch.as_tensor(_f64(x)).to(dev, non_blocking=False)
            sa, ss, rho, T = put(wl.sigma_a), put(wl.sigma_s), put(wl.rho), put(wl.T)
            v = put(np.reshape(wl.v, (3, nc)))
            I = [torch.empty((nang, nc), dtype=sdt, device=dev) for _ in range(2)]
            E = torch.empty(nc, dtype=torch.float64, device=dev)
            F = torch.empty((3, nc), dtype=torch.float64, device=dev)
            tot = torch.empty(rt.RT_NTOT, dtype=torch.float64, device=dev)
            rt.rt_bind_intensity(ctx, I[0], I[1])
            rt.rt_equilibrium_intensity(ctx, T, I[0], stream)
            rt.rt_step(ctx, wl.dt, int(wl.nsteps), rt.make_fields(sa, ss, rho, T, v),
                       rt.make_out(E, F, None, None, None, tot), stream)
            T_h, E_h, F_h, tot_h = T.cpu(), E.cpu(), F.cpu(), tot.cpu()
            st = rt.rt_sync_status(ctx)
        finally:
            rt.rt_destroy(ctx)
        if st != rt.RT_OK:
            raise RuntimeError(f"plain-path request {i} failed: {rt.rt_strerror(st)}")
        done = time.perf_counter()
        t_first = arrive if t_first is None else t_first
        t_last = done
        lat.append(done - arrive)
        classes.append(request_class(wl, nang, packed_cells, large_work))
        work += float(nc) * nang * wl.nsteps
        del T_h, E_h, F_h, tot_h
        if progress and (i + 1) % 50 == 0:
            progress(f"plain path {i + 1}/{len(wls)}")
    out = dict(requests=len(wls), makespan_s=t_last - t_first, updates=work,
               throughput=work / (t_last - t_first))
    out.update({f"latency_{k}_s": v for k, v in _percentiles(lat).items()})
    out["latency_by_class_s"] = _by_class(lat, classes)
    return out
