"""Steady-state pin of the whole oracle step with copy and vacuum faces:
the non-LTE atmosphere of paper Section 5.3.  With one direction per octant
(Eddington closure) the steady state of the transfer equation is
E_r(tau) = 1 - exp(-sqrt(3 eps) tau)/(1 + sqrt(eps)), which the time-dependent
step reaches (here eps = 0.1) to the discretization error of 1280 cells."""
import numpy as np
import pytest

import workloads as W


def test_atmosphere_reaches_the_analytic_steady_state(orc):
    eps = 0.1
    wl = W.atmosphere(eps)
    st = orc.State(orc.Problem(wl)).step(nsteps=8000)
    tau = wl.meta["tau"]
    Ea = 1.0 - np.exp(-np.sqrt(3 * eps) * tau) / (1.0 + np.sqrt(eps))
    sel = (tau > 0.05) & (tau < 50.0)
    assert np.abs(st.E - Ea)[sel].max() <= 2e-3
    assert np.all(st.T == 1.0)               # the temperature is held
    # the top of the atmosphere is darker for smaller eps: E(0) = sqrt(eps)/(1 + sqrt(eps))
    assert abs(st.E[-1] - np.sqrt(eps) / (1 + np.sqrt(eps))) <= 2e-3


def test_atmosphere_setup_is_the_papers():
    """The workload is the printed setup of Section 5.3."""
    from golden_values import golden
    s = golden("sec5_3_atmosphere.json")
    wl = W.atmosphere(0.1)
    assert wl.n[0] == s["cells_z"]
    assert wl.n[0] * wl.dx[0] == pytest.approx(s["box_z"][1] - s["box_z"][0])
    z = s["box_z"][0] + (np.arange(wl.n[0]) + 0.5) * wl.dx[0]
    assert np.allclose(wl.rho, 1e-3 * np.exp(10.0 - z), rtol=1e-14)
    for eps in s["eps_range"]:
        w = W.atmosphere(eps)
        assert np.allclose(w.sigma_a, eps * w.rho) and np.allclose(w.sigma_s, (1 - eps) * w.rho)
