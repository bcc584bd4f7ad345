"""The reduced speed of light (Section 6 reading, rt_params.c_reduced) on
the GPU: parity with the oracle while the temperature evolves, with flow
(O(v/C) terms), absorption and scattering, in both kernels; at fixed
temperature the run at c_r with the step dt C/c_r equals the run at C with
dt (the same radiation step); invalid combinations are rejected."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "mixed": 1e-5}


def _nerr(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    den = np.abs(b).max()
    return float(np.abs(a - b).max() / den) if den > 0 else float(np.abs(a - b).max())


def _cases():
    return dict(
        box3d=W.small_case(3, (10, 9, 8), ("ls", 6), seed=91, vscale=0.03, C=5.0),
        slab_many_angles=W.small_case(1, (48,), ("gl", 330), seed=92, vscale=0.02, C=4.0),
        plane2d=W.small_case(2, (17, 13), ("ls", 8), seed=93, vscale=0.02, kappa_a=3.0,
                             kappa_s=0.5, C=8.0))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name", ["box3d", "slab_many_angles", "plane2d"])
def test_reduced_speed_matches_oracle(name, precision):
    import oracle

    from paper_1403_6126_amd.solver import Solver
    wl = _cases()[name]
    cr = wl.C / 4.0
    wl.courant *= 2.0      # the radiation's Courant number is half the workload's
    nsteps = 6
    ref = oracle.State(oracle.Problem(wl, estimate_v=False, c_reduced=cr)).step(nsteps=nsteps)
    s = Solver(wl, precision=precision, estimate_v=False, c_reduced=cr)
    print(f"case {wl.name} {precision}: c_r = C/4, {nsteps} steps", flush=True)
    s.step(nsteps)
    st = s.state()
    status = s.status()
    s.close()
    assert status == 0
    errs = {k: _nerr(st[k], r) for k, r in (("I", ref.I), ("T", ref.T), ("E", ref.E),
                                           ("F", ref.F), ("dEgas", ref.dEgas),
                                           ("dMom", ref.dMom))}
    print("   errors", errs, flush=True)
    tol = TOL[precision]
    assert max(errs.values()) <= tol, errs


def test_reduced_speed_longer_step_at_fixed_temperature():
    from paper_1403_6126_amd.solver import Solver
    a = W.atmosphere(0.1)
    b = W.atmosphere(0.1)
    b.courant = a.courant * 4.0
    sa_ = Solver(a, estimate_v=False)
    sb_ = Solver(b, estimate_v=False, c_reduced=b.C / 4.0)
    sa_.step(2000)
    sb_.step(2000)
    ea, eb = sa_.state(), sb_.state()
    sa_.close()
    sb_.close()
    err = _nerr(eb["E"], ea["E"])
    print(f"atmosphere eps=0.1, 2000 steps: c_r = C/4 at 4 dt against C at dt: E {err:.2e}",
          flush=True)
    assert err <= 1e-12 and np.all(eb["T"] == 1.0)


def test_reduced_speed_arguments():
    from paper_1403_6126_amd import rt
    from paper_1403_6126_amd.solver import Solver
    wl = W.small_case(2, (6, 5), ("ls", 4), seed=94, C=4.0)
    for kw, status in ((dict(c_reduced=2.0), rt.RT_EUNSUPPORTED),             # with the estimate
                       (dict(c_reduced=5.0, estimate_v=False), rt.RT_EINVAL),   # above C
                       (dict(c_reduced=-1.0, estimate_v=False), rt.RT_EINVAL)):
        with pytest.raises(rt.RTError) as e:
            Solver(wl, **kw)
        assert e.value.status == status
    # the CFL limit is that of the reduced speed: sum_d c_r |mu_d| dt/dx_d <= 1
    from paper_1403_6126_amd.solver import quadrature_for
    mu, _ = quadrature_for(wl.quad)
    lim = 1.0 / (1.0 * max(abs(m[0]) / wl.dx[0] + abs(m[1]) / wl.dx[1] for m in mu))
    s = Solver(wl, estimate_v=False, c_reduced=1.0)
    try:
        s.step(1, dt=0.99 * lim)           # four times the limit of the full speed C = 4
        assert s.status() == 0
        with pytest.raises(rt.RTError) as e:
            s.step(1, dt=1.01 * lim)
        assert e.value.status == rt.RT_ECFL
    finally:
        s.close()
