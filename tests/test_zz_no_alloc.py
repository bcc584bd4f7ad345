"""rt_step_static (the entry point that allocates nothing: its library
scratch is a file-scope device array) against rt_create + rt_step on the
same inputs, on two calls in a row, the second with a smaller grid, and its
size limit.  The results must agree to the FP64 bar (they run the same
kernels, so they agree bit for bit)."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _plain(wl, nsteps):
    from paper_1403_6126_amd.solver import Solver
    s = Solver(wl)
    s.step(nsteps)
    st = s.state()
    assert s.status() == 0
    s.close()
    return st


def _static(wl, nsteps):
    import torch

    from paper_1403_6126_amd import rt
    from paper_1403_6126_amd.solver import quadrature_for
    mu, w = quadrature_for(wl.quad)
    dev = torch.device("cuda")
    f64 = dict(dtype=torch.float64, device=dev)
    put = lambda a: torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).to(dev)
    nc = wl.ncell
    sa, ss, rho, T = put(wl.sigma_a), put(wl.sigma_s), put(wl.rho), put(wl.T)
    v = put(wl.v).reshape(3, nc).contiguous()
    Ia = put(wl.init(mu))
    Ib = torch.empty_like(Ia)
    E, F, P = torch.zeros(nc, **f64), torch.zeros((3, nc), **f64), torch.zeros((6, nc), **f64)
    dEgas, dMom = torch.zeros(nc, **f64), torch.zeros((3, nc), **f64)
    tot = torch.zeros(rt.RT_NTOT, **f64)
    status = torch.zeros(1, dtype=torch.int32, device=dev)
    grid = rt.make_grid(wl.ndim, wl.n, wl.dx, wl.bc)
    params = rt.make_params(wl.C, wl.P, wl.gamma, wl.R, rt.RT_FP64, rt.RT_ESTIMATE_V)
    rt.rt_step_static(grid, mu, w, params, Ia, Ib, wl.dt, nsteps,
                      rt.make_fields(sa, ss, rho, T, v), rt.make_out(E, F, P, dEgas, dMom, tot),
                      status, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    assert int(status.item()) == 0
    I = (Ib if nsteps % 2 else Ia).cpu().numpy()
    return dict(I=I, T=T.cpu().numpy(), E=E.cpu().numpy(), F=F.cpu().numpy(),
                P=P.cpu().numpy(), dEgas=dEgas.cpu().numpy(), dMom=dMom.cpu().numpy(),
                totals=tot.cpu().numpy())


def _nerr(a, b):
    den = np.abs(b).max()
    return float(np.abs(a - b).max() / den) if den > 0 else float(np.abs(a - b).max())


def test_static_scratch_matches_context_path():
    cases = [W.small_case(3, (40, 36, 30), ("ls", 8), seed=81, vscale=0.03, kappa_s=3.0),
             W.small_case(3, (12, 10, 9), ("ls", 4), seed=82, vscale=0.05, kappa_a=2.0)]
    for wl in cases:                     # the second call has the smaller grid
        nsteps = 5
        print(f"case {wl.name} ncell={wl.ncell} steps={nsteps}", flush=True)
        a = _static(wl, nsteps)
        b = _plain(wl, nsteps)
        errs = {k: _nerr(a[k], b[k]) for k in ("I", "T", "E", "F", "P", "dEgas", "dMom")}
        print("   rt_step_static vs rt_step", errs, flush=True)
        assert max(errs.values()) <= 1e-12, errs


def test_static_scratch_rejects_too_large():
    import torch

    from paper_1403_6126_amd import rt
    wl = W.small_case(3, (64, 64, 64), ("ls", 4), seed=83)
    with pytest.raises(rt.RTError) as e:
        _static(wl, 1)
    assert e.value.status == rt.RT_ETOOBIG
    torch.cuda.synchronize()
