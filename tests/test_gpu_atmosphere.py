"""The non-LTE atmosphere (paper Section 5.3) on the GPU: the time-dependent
step reaches the analytic steady state E_r(tau) = 1 - exp(-sqrt(3 eps) tau)
/ (1 + sqrt(eps)) for eps from 0.1 to 1e-4 (copy and vacuum faces, one
direction per octant), and matches the oracle along the way."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("eps,nsteps,tol", [(0.1, 16000, 2e-3), (1e-2, 32000, 3e-3),
                                            (1e-3, 100000, 5e-3), (1e-4, 200000, 1e-2)])
def test_atmosphere_steady_state(eps, nsteps, tol):
    from paper_1403_6126_amd.solver import Solver
    wl = W.atmosphere(eps)
    s = Solver(wl)
    s.step(nsteps)
    st = s.state()
    status = s.status()
    s.close()
    assert status == 0
    tau = wl.meta["tau"]
    Ea = 1.0 - np.exp(-np.sqrt(3 * eps) * tau) / (1.0 + np.sqrt(eps))
    sel = (tau > 0.05) & (tau < 50.0)
    err = float(np.abs(st["E"] - Ea)[sel].max())
    print(f"atmosphere eps={eps}: {nsteps} steps, max |E - E_analytic| (0.05 < tau < 50) {err:.2e}, "
          f"E(top) {st['E'][-1]:.4f} vs {np.sqrt(eps) / (1 + np.sqrt(eps)):.4f}", flush=True)
    assert err <= tol
    assert np.all(st["T"] == 1.0)


def test_atmosphere_matches_oracle():
    import oracle

    from paper_1403_6126_amd.solver import Solver
    wl = W.atmosphere(0.1)
    ref = oracle.State(oracle.Problem(wl)).step(nsteps=1000)
    s = Solver(wl)
    s.step(1000)
    st = s.state()
    s.close()
    err = float(np.abs(st["E"] - ref.E).max() / np.abs(ref.E).max())
    errI = float(np.abs(st["I"] - ref.I).max() / np.abs(ref.I).max())
    print(f"atmosphere eps=0.1, 1000 steps, FP64 vs oracle: E {err:.2e}, I {errI:.2e}", flush=True)
    assert max(err, errI) <= 1e-12
