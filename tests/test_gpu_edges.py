"""Degenerate and extreme inputs on the GPU against the oracle: a one-cell
periodic slab (every stencil neighbour is the cell itself), a single-cell
axis inside a 3D grid, pure transport without opacity from a non-equilibrium
start, the largest angle set the library accepts (1024 directions, the
thread-per-cell kernel), a cold optically thick gas, and a call of zero
steps.  FP64 within 1e-12 normwise, FP32-mixed within 1e-5."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "mixed": 1e-5}


def _nerr(a, b):
    den = np.abs(b).max()
    return float(np.abs(a - b).max() / den) if den > 0 else float(np.abs(a - b).max())


def _random_init(wl, seed):
    def init(mu, seed=seed, nc=wl.ncell):
        g = np.random.Generator(np.random.PCG64(seed))
        return g.uniform(0.05, 1.0, (np.asarray(mu).shape[0], nc))
    wl.init = init
    return wl


def _check(wl, nsteps, precision):
    import oracle

    from paper_1403_6126_amd.solver import Solver
    ref = oracle.run(wl, nsteps=nsteps)
    s = Solver(wl, precision=precision)
    print(f"case {wl.name} nang={s.nang} ncell={wl.ncell} steps={nsteps} {precision}", flush=True)
    s.step(nsteps)
    st = s.state()
    status = s.status()
    s.close()
    assert status == 0
    errs = {k: _nerr(st[k], r) for k, r in
            (("I", ref.I), ("T", ref.T), ("E", ref.E), ("F", ref.F), ("P", ref.Pr))}
    print("   errors", errs, flush=True)
    assert max(errs.values()) <= TOL[precision], errs


def _cases():
    one = W.small_case(1, (1,), ("gl", 4), seed=71, vscale=0.01, kappa_a=2.0, kappa_s=1.0)
    flat = W.small_case(3, (6, 1, 5), ("ls", 4), seed=72, vscale=0.03)
    free = _random_init(W.small_case(2, (17, 9), ("ls", 6), seed=73, kappa_a=0.0,
                                     kappa_s=0.0, vscale=0.0), 74)
    wide = W.small_case(1, (40,), ("gl", 1024), seed=75, vscale=0.01, courant=0.3)
    cold = W.small_case(3, (9, 7, 6), ("ls", 8), seed=76, kappa_a=50.0, kappa_s=5.0,
                        T_s=0.1, vscale=0.01)
    cold.T *= 0.05
    cold.init = lambda mu, T=cold.T: W.equilibrium_intensity(T, np.asarray(mu).shape[0])
    return dict(one_cell=one, single_cell_axis=flat, pure_transport=free, max_angles=wide,
                cold_thick=cold)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name", ["one_cell", "single_cell_axis", "pure_transport", "max_angles",
                                  "cold_thick"])
def test_edge_case(name, precision):
    wl = _cases()[name]
    _check(wl, 5, precision)


def test_zero_steps_is_a_no_op():
    from paper_1403_6126_amd.solver import Solver
    wl = W.small_case(3, (10, 9, 8), ("ls", 4), seed=77)
    s = Solver(wl)
    I0 = s.current().double().cpu().numpy().copy()
    T0 = s.T.cpu().numpy().copy()
    s.step(0)
    st = s.state()
    s.close()
    assert np.array_equal(st["I"], I0) and np.array_equal(st["T"], T0)


def test_fixed_table_upload_is_ordered_after_queued_steps():
    # rt_set_fixed_bc called while steps are still queued on a non-blocking
    # stream: those steps read the old inflow table, the later ones the new
    # table.  The oracle takes the same sequence.
    import torch

    import oracle
    from paper_1403_6126_amd import rt
    from paper_1403_6126_amd.solver import Solver
    bc = ((W.BC_FIXED, W.BC_FIXED), (W.BC_PERIODIC, W.BC_PERIODIC), (W.BC_COPY, W.BC_VACUUM))
    wl = W.small_case(3, (40, 24, 20), ("ls", 4), seed=78, vscale=0.02, bc=bc, ghost_seed=9)
    n1, n2 = 40, 5
    mu = oracle.Problem(wl).mu
    tabs = wl.ghost(mu)
    new_tab = 3.0 * tabs[(0, 0)] + 0.5
    a = oracle.run(wl, nsteps=n1)
    tabs_b = dict(tabs)
    tabs_b[(0, 0)] = new_tab
    b = oracle.State(oracle.Problem(wl, ghost=tabs_b), I0=a.I, T0=a.T).step(nsteps=n2)
    stream = torch.cuda.Stream()
    s = Solver(wl)
    torch.cuda.synchronize()                         # the uploads of the set-up
    with torch.cuda.stream(stream):
        s.step(n1)                                   # queued, not waited for
        rt.rt_set_fixed_bc(s.ctx, 0, 0, new_tab)     # host call while they run
        s.step(n2)
    stream.synchronize()
    st = s.state()
    status = s.status()
    s.close()
    assert status == 0
    errs = {k: _nerr(st[k], r) for k, r in (("I", b.I), ("T", b.T), ("E", b.E))}
    print("   errors", errs, flush=True)
    assert max(errs.values()) <= TOL["fp64"], errs
