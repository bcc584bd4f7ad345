"""Gas feedback pin (paper Section 5.2, equilibrium in a moving medium).

A uniform periodic 2D medium (rho = T = 1, E_r = 1, isotropic I, Prat = 1,
Crat = 10, three directions per octant) is given v_x = 0.3 Crat, and the
momentum exchange of every step moves the gas (rho fixed).  The paper
reports, for sigma_a = 100: the comoving flux vanishes in equilibrium
(F_r = F_v = v_x (E_r + P_xx)/Crat), rho v_x + Prat F_r/Crat is conserved,
f_xx = P_xx/E_r rises to about 0.37 while f_yy falls to about 0.315, and the
total energy error is about 1e-4; for sigma_s = 100 the same, with the gas
temperature unchanged.
"""
import numpy as np
import pytest

import workloads as W
from golden_values import golden


def _setup(sa, ss, vx=3.0):
    wl = W.small_case(2, (2, 2), ("ls", 4), seed=1, courant=0.4, C=10.0, P=1.0, kappa_a=0,
                      kappa_s=0, vscale=0)
    wl.dx = (1 / 32, 1 / 32, 1.0)
    wl.rho[:] = 1
    wl.T[:] = 1
    wl.v[:] = 0
    wl.v[0] = vx
    wl.sigma_a[:] = sa
    wl.sigma_s[:] = ss
    wl.init = lambda mu, nc=wl.ncell: np.full((np.asarray(mu).shape[0], nc), 1 / (4 * np.pi))
    return wl


def _diag(st, wl):
    E, Fx, Pxx, Pyy = st.E.mean(), st.F[0].mean(), st.Pr[0].mean(), st.Pr[1].mean()
    v = st.v[0].mean()
    cv = wl.R / (wl.gamma - 1)
    return dict(fxx=Pxx / E, fyy=Pyy / E, F=Fx, Fv=v * (E + Pxx) / wl.C, T=st.T.mean(),
                mom=v + wl.P * Fx / wl.C,
                energy=cv * st.T.mean() + 0.5 * (st.v ** 2).sum(0).mean() + wl.P * E)


@pytest.mark.parametrize("sa,ss", [(100.0, 0.0), (0.0, 100.0)])
def test_moving_medium_equilibrium(orc, sa, ss):
    g = golden("sec5_2_moving_medium.json")
    wl = _setup(sa, ss, vx=g["v_x_over_Crat"] * 10.0)
    st = orc.State(orc.Problem(wl, feedback=True))
    d0 = _diag(st, wl)
    assert abs(d0["fxx"] - g["f_initial"]) <= 1e-12                # isotropic start
    st.step(nsteps=100)
    d = _diag(st, wl)
    # the printed equilibrium (about 0.37 and 0.315: two printed digits)
    assert abs(d["fxx"] - g["f_xx_equilibrium_about"]) <= 0.005, d
    assert abs(d["fyy"] - g["f_yy_equilibrium_about"]) <= 0.005, d
    assert abs(d["F"] - d["Fv"]) <= 1e-6 * d["Fv"], d            # comoving flux gone
    assert abs(d["mom"] - d0["mom"]) <= 1e-13 * d0["mom"]         # momentum conserved
    assert abs(d["energy"] - d0["energy"]) <= g["relative_energy_error_about"] * d0["energy"]
    assert st.v[0].mean() < 3.0                                    # the gas was dragged
    if sa == 0.0:
        assert np.all(st.T == 1.0)                                 # scattering: T unchanged


def test_without_feedback_the_gas_is_not_dragged(orc):
    wl = _setup(100.0, 0.0)
    st = orc.State(orc.Problem(wl))
    st.step(nsteps=20)
    assert np.all(st.v[0] == 3.0)
