"""Pins of the oracle's transport step (paper Section 4.2)."""
import numpy as np
import pytest

import workloads as W
from oracle import dense
from oracle.quadrature import level_symmetric, gauss_legendre


def _wl(ndim, shape, quad, bc=None, C=1.0, courant=0.4, seed=5, sig=1.0, vs=0.02):
    return W.small_case(ndim, shape, quad, seed=seed, courant=courant, kappa_a=0.3 * sig,
                        kappa_s=sig, vscale=vs, bc=bc, C=C)


def _rand_state(orc, wl, seed=9):
    prob = orc.Problem(wl)
    rng = np.random.default_rng(seed)
    I = rng.uniform(0.1, 1.0, (prob.nang, wl.ncell))
    E, F, Pr = orc.moments(prob, I)
    return prob, I, E / (4 * np.pi)


def test_uniform_intensity_gives_zero_increment(orc):
    wl = _wl(3, (6, 5, 4), ("ls", 4))
    nc = wl.ncell
    wl.v[:] = np.array([0.01, -0.02, 0.005])[:, None]
    wl.sigma_a[:] = 0.7
    wl.sigma_s[:] = 2.0
    prob = orc.Problem(wl)
    I = np.full((prob.nang, nc), 0.3)
    J = np.full(nc, 0.3)
    dF = orc.transport(prob, wl.dt, I, J, wl.v, wl.sigma_a, wl.sigma_s)
    assert np.all(dF == 0.0)


@pytest.mark.parametrize("ndim,shape,quad", [(1, (37,), ("gl", 8)), (2, (9, 7), ("ls", 4)),
                                             (3, (6, 5, 7), ("ls", 6))])
def test_periodic_conservation_per_ray(orc, ndim, shape, quad):
    # interface fluxes are single valued, so sum over cells of Delta F_m is
    # zero to round-off for every angle (Section 4.2)
    wl = _wl(ndim, shape, quad)
    prob, I, J = _rand_state(orc, wl)
    dF = orc.transport(prob, wl.dt, I, J, wl.v, wl.sigma_a, wl.sigma_s)
    tot = dF.sum(axis=1)
    scale = np.abs(dF).sum(axis=1)
    assert np.all(np.abs(tot) <= 1e-14 * scale + 1e-300)
    assert np.abs(dF).max() > 0


def _axis_table(ndim):
    # directions along the axes; power-of-two weights
    if ndim == 1:
        mu = np.array([[1.0, 0, 0], [-1.0, 0, 0]])
        w = np.array([0.5, 0.5])
    else:
        mu = np.array([[1.0, 0, 0], [-1.0, 0, 0], [0, 1.0, 0], [0, -1.0, 0],
                       [0, 0, 1.0], [0, 0, -1.0]])
        w = np.array([0.25, 0.25, 0.125, 0.125, 0.125, 0.125])
    return mu, w


@pytest.mark.parametrize("ndim,shape", [(1, (16,)), (3, (8, 6, 5))])
def test_exact_shift_at_courant_one(orc, ndim, shape):
    # vacuum, v = 0, C |mu| dt / dx = 1: a 0/1 top hat moves one cell per step
    # along every axis direction, bitwise, and returns after n steps
    mu, w = _axis_table(ndim)
    wl = W.small_case(ndim, shape, ("table", mu, w), courant=1.0, kappa_a=0.0,
                      kappa_s=0.0, vscale=0.0)
    wl.dx = (1.0, 1.0, 1.0)
    assert wl.dt == 1.0
    nc = wl.ncell
    n = wl.n
    rng = np.random.default_rng(3)
    base = (rng.uniform(size=(len(w), n[2], n[1], n[0])) > 0.6).astype(float)
    prob = orc.Problem(wl, mu, w)
    st = orc.State(prob, I0=base.reshape(len(w), nc), T0=np.ones(nc))
    st.step(dt=1.0)
    got = st.I.reshape(base.shape)
    for m in range(len(w)):
        d = int(np.argmax(np.abs(mu[m])))
        s = int(np.sign(mu[m, d]))
        exp = np.roll(base[m], s, axis=2 - d)
        assert np.array_equal(got[m], exp), m
    st.step(dt=1.0, nsteps=int(np.lcm.reduce([n[d] for d in range(ndim)])) - 1)
    assert np.array_equal(st.I.reshape(base.shape), base)


def test_mirror_symmetry(orc):
    # reflecting x -> -x (cells reversed, mu_x and v_x negated) mirrors Delta F
    wl = _wl(3, (7, 5, 4), ("ls", 6), vs=0.05)
    prob, I, J = _rand_state(orc, wl)
    mu = prob.mu
    n = wl.n
    perm = np.array([int(np.argmin(np.abs(mu - mu[m] * np.array([-1, 1, 1])).sum(1)))
                     for m in range(len(mu))])
    assert np.array_equal(mu[perm], mu * np.array([-1, 1, 1]))

    def flip(a):  # reverse along x of a (..., ncell) array
        return np.ascontiguousarray(a.reshape(a.shape[:-1] + (n[2], n[1], n[0]))[..., ::-1]
                                    .reshape(a.shape))

    dF = orc.transport(prob, wl.dt, I, J, wl.v, wl.sigma_a, wl.sigma_s)
    v2 = flip(wl.v)
    v2[0] *= -1
    dF2 = orc.transport(prob, wl.dt, flip(I[perm]), flip(J), v2, flip(wl.sigma_a),
                       flip(wl.sigma_s))
    assert np.array_equal(dF2, flip(dF[perm]))


def test_linear_profile_moves_nu_cells(orc):
    # a linear ramp in I (v = 0) is advanced exactly by nu cells per step in
    # the interior, for any alpha
    mu, w = _axis_table(1)
    for sig in (0.0, 30.0):
        wl = W.small_case(1, (24,), ("table", mu, w), courant=0.4, kappa_a=0.0, kappa_s=0.0,
                          vscale=0.0)
        wl.sigma_s[:] = sig
        prob = orc.Problem(wl, mu, w)
        x = np.arange(24.0)
        I = np.vstack([2.0 + 0.1 * x, 5.0 - 0.2 * x])
        dF = orc.transport(prob, wl.dt, I, np.zeros(24), wl.v, wl.sigma_a, wl.sigma_s)
        nu = wl.C * wl.dt / wl.dx[0]
        inner = slice(3, 21)
        assert np.allclose(dF[0, inner], -nu * 0.1, rtol=1e-12)
        assert np.allclose(dF[1, inner], -nu * 0.2, rtol=1e-12)


def test_second_order_convergence_smooth_advection(orc):
    # vacuum advection of a smooth periodic profile for one period: the van
    # Leer piecewise-linear scheme converges at close to second order (a
    # first-order upwind flux would give order 1)
    mu, w = _axis_table(1)
    errs = []
    for nx in (32, 64, 128, 256):
        wl = W.small_case(1, (nx,), ("table", mu, w), courant=0.5, kappa_a=0.0, kappa_s=0.0,
                          vscale=0.0)
        x = (np.arange(nx) + 0.5) / nx
        I0 = 1.0 + 0.5 * np.sin(2 * np.pi * x)
        prob = orc.Problem(wl, mu, w)
        st = orc.State(prob, I0=np.vstack([I0, I0]), T0=np.ones(nx))
        st.step(nsteps=2 * nx)                  # t = 1 at courant 0.5
        errs.append(np.abs(st.I[0] - I0).mean())
    order = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(order > 1.6), order


@pytest.mark.parametrize("ndim,shape,quad", [(1, (11,), ("gl", 4)), (2, (5, 4), ("ls", 2)),
                                             (3, (4, 3, 5), ("ls", 4))])
def test_against_vectorised_periodic_transport(orc, ndim, shape, quad):
    wl = _wl(ndim, shape, quad, vs=0.05, sig=20.0)
    prob, I, J = _rand_state(orc, wl)
    dF = orc.transport(prob, wl.dt, I, J, wl.v, wl.sigma_a, wl.sigma_s)
    n = wl.n
    sh = (n[2], n[1], n[0])
    ref = dense.transport_periodic(sh, wl.dx[:ndim], prob.mu, wl.C, wl.dt,
                                   I.reshape((-1,) + sh), J.reshape(sh), wl.v.reshape((3,) + sh),
                                   wl.sigma_a.reshape(sh), wl.sigma_s.reshape(sh))
    ref = ref.reshape(dF.shape)
    assert np.abs(dF - ref).max() <= 1e-13 * np.abs(ref).max()


def test_fixed_boundary_inflow(orc):
    # vacuum, courant 1, fixed ghost table: the inflow value enters the first
    # cell after one step and travels one cell per step
    mu, w = _axis_table(1)
    wl = W.small_case(1, (8,), ("table", mu, w), courant=1.0, kappa_a=0.0, kappa_s=0.0,
                      vscale=0.0, bc=((W.BC_FIXED, W.BC_FIXED), (0, 0), (0, 0)))
    wl.dx = (1.0, 1.0, 1.0)
    ghost = {(0, 0): np.array([4.0, 0.0]), (0, 1): np.array([0.0, 2.0])}
    prob = orc.Problem(wl, mu, w, ghost=ghost)
    st = orc.State(prob, I0=np.zeros((2, 8)), T0=np.ones(8))
    for k in range(1, 9):
        st.step(dt=1.0)
        assert np.array_equal(st.I[0, :k], np.full(k, 4.0)) and np.all(st.I[0, k:] == 0)
        assert np.array_equal(st.I[1, 8 - k:], np.full(k, 2.0)) and np.all(st.I[1, :8 - k] == 0)
