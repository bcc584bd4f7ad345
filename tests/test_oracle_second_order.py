"""Pins of the second-order-in-time absorption step of the oracle (Section
4.3: the gas energy change of the first-order step differs from the
radiation energy change at O(dt^2); solving the absorption system twice
reduces that gap).

The pin is energy conservation itself, which the oracle does not enforce:
on a uniform periodic box (no transport) with pure absorption, the total
energy error of one step, sum(dE_gas) + P sum(dE_r), must fall as dt^2 for
the single solve and at least as dt^2.6 for the second-order solve, and be
far smaller.  A slip in the time-centred velocity (the full momentum change
instead of half of it, a sign) leaves an O(dt^2) error and fails here."""
import math

import numpy as np
import pytest

import oracle
from workloads.configs import Workload

FOURPI = 4.0 * math.pi


def uniform_box(sa=5.0, ss=0.0, v=(0.3, -0.2, 0.1), C=10.0, P=1.0, n=4, order=4, seed=0):
    nc = n ** 3
    wl = Workload(name="uniform-absorbing-box", n=(n, n, n), ndim=3, dx=(1.0 / n,) * 3,
                  bc=((0, 0), (0, 0), (0, 0)), quad=("ls", order), C=C, P=P, courant=0.4,
                  rho=np.ones(nc), T=np.ones(nc), v=np.tile(np.asarray(v, float)[:, None], nc),
                  sigma_a=np.full(nc, sa), sigma_s=np.full(nc, ss))
    def init(mu, seed=seed):
        rng = np.random.default_rng(seed)
        aniso = 1.5 + 0.8 * rng.random(np.asarray(mu).shape[0])
        return np.repeat((aniso / FOURPI)[:, None], nc, axis=1)
    wl.init = init
    return wl


def energy_error(wl, dt, **kw):
    prob = oracle.Problem(wl, **kw)
    st = oracle.State(prob)
    E0 = st.E.copy()
    st.step(dt=dt)
    return float(np.sum(st.dEgas) + wl.P * np.sum(st.E - E0)) * wl.cell_volume, st


@pytest.mark.parametrize("estimate_v", [False, True])
def test_energy_error_order(estimate_v):
    wl = uniform_box()
    dts = [2.5e-3, 1.25e-3]
    e1 = [energy_error(wl, dt, estimate_v=estimate_v)[0] for dt in dts]
    e2 = [energy_error(wl, dt, estimate_v=estimate_v, second_order=True)[0] for dt in dts]
    order1 = math.log2(abs(e1[0] / e1[1]))
    order2 = math.log2(abs(e2[0] / e2[1]))
    assert 1.7 < order1 < 2.3, order1
    assert order2 > 2.6, order2
    assert abs(e2[1]) < 1e-2 * abs(e1[1]), (e1, e2)


def test_no_coupling_is_single_solve():
    # P = 0: the radiation exchanges no momentum with the gas, the centred
    # velocity is v itself, and the second solve repeats the first
    wl = uniform_box(P=0.0)
    _, a = energy_error(wl, 2e-3, estimate_v=False)
    _, b = energy_error(wl, 2e-3, estimate_v=False, second_order=True)
    assert np.array_equal(a.I, b.I) and np.array_equal(a.T, b.T)


def test_momentum_still_conserved():
    # the momentum exchange is taken from the conservation of gas plus
    # radiation momentum, with either solve
    wl = uniform_box(ss=2.0)
    _, st = energy_error(wl, 2e-3, second_order=True)
    prob = st.prob
    E0, F0, _ = oracle.moments(prob, wl.init(prob.mu))
    rad = wl.P / wl.C * (st.F - F0)
    assert np.max(np.abs(st.dMom + rad)) < 1e-13 * np.max(np.abs(rad))


def test_scattering_energy_unchanged():
    # scattering keeps the step's velocity: with no absorption the two
    # schemes are the same step
    wl = uniform_box(sa=0.0, ss=3.0)
    _, a = energy_error(wl, 2e-3)
    _, b = energy_error(wl, 2e-3, second_order=True)
    assert np.array_equal(a.I, b.I) and np.array_equal(a.T, b.T)


def test_energy_error_order_reduced_speed():
    # with a reduced speed of light c_hat the gas sees C/c_hat times the
    # radiation's momentum change, and the centred velocity takes the gas's
    # change; the conserved energy is (C/c_hat) P E_r + e_gas
    wl = uniform_box()
    chat = wl.C / 4.0

    def err(dt, **kw):
        prob = oracle.Problem(wl, estimate_v=False, c_reduced=chat, **kw)
        st = oracle.State(prob)
        E0 = st.E.copy()
        st.step(dt=dt)
        return float(np.sum(st.dEgas) + wl.C / chat * wl.P * np.sum(st.E - E0)) * wl.cell_volume
    dts = [1e-2, 5e-3]
    e1 = [err(dt) for dt in dts]
    e2 = [err(dt, second_order=True) for dt in dts]
    o1, o2 = math.log2(abs(e1[0] / e1[1])), math.log2(abs(e2[0] / e2[1]))
    assert 1.5 < o1 < 2.3, o1
    assert o2 > 2.6, o2
    assert abs(e2[1]) < 1e-2 * abs(e1[1]), (e1, e2)
