"""Oracle pins for the reduced speed of light combined with the method
(Section 6; reading: the radiation advances at c_r <= C in its transport
and both implicit source steps, the gas exchanges energy and momentum at the
true rate, the O(v/C) factors keep C).

* Section 5.1 (uniform static medium) with c_r = C/10: every step is the
  backward-Euler step of dE/dt = c_r sigma (T^4 - E), c_v dT/dt = -P C sigma
  (T^4 - E), whose closed form gives c_v T' + k T'^4 = c_v T + k E with
  k = P C sigma dt / (1 + c_r sigma dt); (C/c_r) P E + c_v T is conserved and
  the equilibrium is the root of (C/c_r) P T^4 + c_v T = (C/c_r) P E0 + c_v T0,
  not that of the full speed.
* With the temperature held fixed the radiation alone evolves: the run at
  c_r with the step dt C/c_r is the run at C with dt (same radiation step),
  so their intensities agree to rounding at every step.
* c_r = C is the method itself, bit for bit."""
import numpy as np
import pytest

import workloads as W
from golden_values import golden

FOUR_PI = 4.0 * np.pi


@pytest.fixture(scope="module")
def orc():
    import oracle
    return oracle


def _uniform(orc, sa, E0, T0, cr):
    wl = W.small_case(2, (8, 8), ("ls", 4), seed=1, courant=0.4, C=10.0, P=1.0,
                      kappa_a=0.0, kappa_s=0.0, vscale=0.0)
    wl.rho[:] = 1.0
    wl.T[:] = T0
    wl.sigma_a[:] = sa
    prob = orc.Problem(wl, estimate_v=False, c_reduced=cr)
    st = orc.State(prob, I0=np.full((prob.nang, wl.ncell), E0 / FOUR_PI),
                   T0=np.full(wl.ncell, T0))
    return wl, st


def _root(a, b, rhs):
    roots = np.roots([a, 0, 0, b, -rhs])
    return max(r.real for r in roots if abs(r.imag) < 1e-9 * abs(r) and r.real > 0)


_S51 = golden("sec5_1_thermal_equilibrium.json")


@pytest.mark.parametrize("sa", _S51["sigma_a"])
@pytest.mark.parametrize("E0,T0", [(s["E_r"], s["T4"] ** 0.25) for s in _S51["initial_states"]])
def test_reduced_speed_relaxation_closed_form(orc, sa, E0, T0):
    cr = 1.0
    wl, st = _uniform(orc, sa, E0, T0, cr)
    C, P, dt = wl.C, wl.P, wl.dt
    cv = 1.0 / (5 / 3 - 1)
    k = P * C * sa * dt / (1 + cr * sa * dt)
    E, T = E0, T0
    inv0 = (C / cr) * P * E0 + cv * T0
    for n in range(40):
        st.step()
        Tn = _root(k, cv, cv * T + k * E)
        E = (E + cr * dt * sa * Tn ** 4) / (1 + cr * dt * sa)
        T = Tn
        assert np.allclose(st.E, E, rtol=1e-11)
        assert np.allclose(st.T, T, rtol=1e-11)
        inv = (C / cr) * P * st.E[0] + cv * st.T[0]
        assert abs(inv - inv0) <= 1e-10 * inv0
    Teq = _root((C / cr) * P, cv, inv0)
    Tfull = _root(P, cv, P * E0 + cv * T0)
    assert abs(Teq - Tfull) > 5e-3 * Tfull      # a different equilibrium from the full speed
    if sa == 100.0:
        assert abs(T - Teq) <= 1e-3 * Teq and abs(E - Teq ** 4) <= 1e-3 * Teq ** 4
        assert abs(st.T[0] - Teq) <= 1e-3 * Teq


def test_reduced_speed_is_a_longer_radiation_step_at_fixed_temperature(orc):
    # shadow geometry (Section 5.8) on 32 x 16 cells: T held fixed, no flow
    a = W.shadow2d(nx=32, ny=16, nsteps=40)
    b = W.shadow2d(nx=32, ny=16, nsteps=40)
    cr = a.C / 4.0
    b.courant = a.courant * 4.0            # dt_b = 4 dt_a: the same radiation step
    sa = orc.State(orc.Problem(a, estimate_v=False))
    sb = orc.State(orc.Problem(b, estimate_v=False, c_reduced=cr))
    for n in range(4):
        sa.step(nsteps=10)
        sb.step(nsteps=10)
        err = np.abs(sb.I - sa.I).max() / np.abs(sa.I).max()
        assert err <= 1e-13, (n, err)
    assert np.array_equal(sb.T, a.T) and np.array_equal(sa.T, a.T)


def test_full_speed_is_the_method(orc):
    wl = W.small_case(3, (5, 4, 6), ("ls", 4), seed=5, vscale=0.0)
    s0 = orc.State(orc.Problem(wl, estimate_v=False)).step(nsteps=3)
    s1 = orc.State(orc.Problem(wl, estimate_v=False, c_reduced=wl.C)).step(nsteps=3)
    assert np.array_equal(s0.I, s1.I) and np.array_equal(s0.T, s1.T)
    assert np.array_equal(s0.dMom, s1.dMom) and np.array_equal(s0.dEgas, s1.dEgas)
    with pytest.raises(ValueError):
        orc.Problem(wl, estimate_v=True, c_reduced=0.5 * wl.C)
