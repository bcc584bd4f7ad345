"""Dense brute-force forms of the implicit source steps and a vectorised
periodic transport (TEST INFRASTRUCTURE ONLY).

These solve the paper's equations in their plain, unreduced form with
``numpy.linalg.solve`` and serve to pin the C oracle's O(N) algebra:

* absorption (Section 4.3, Eq. absorptionmatrix): Newton-Raphson on all
  N + 1 unknowns with the full dense Jacobian;
* scattering (Section 4.4): the N x N matrix M_s assembled entry by entry;
* transport (Section 4.2): the interface fluxes on a periodic grid computed
  with whole-array shifts instead of per-cell loops.
"""
from __future__ import annotations

import numpy as np

FOUR_PI = 4.0 * np.pi


def absorption_dense(mu, w, C, P, gamma, R, dt, sa, rho, u, r, Tn, tol=1e-14, maxit=100):
    mu = np.asarray(mu, float)
    w = np.asarray(w, float)
    u = np.asarray(u, float)
    r = np.asarray(r, float)
    N = len(w)
    t = mu @ u
    uu = float(u @ u)
    cv = rho * R / (gamma - 1.0)
    x = np.concatenate([r.copy(), [Tn]])

    def residual(x):
        I, T = x[:N], x[N]
        X = T ** 4 / FOUR_PI
        J = w @ I
        # Eq. absorptionmatrix, first line, times dt
        rhs = (C * sa * (X - I) + 3 * t * sa * X + t * sa * I - sa * uu / C * J
               - sa / C * (w * t * t) @ I)
        G = I - r - dt * rhs
        Hvec = (w * I) @ mu                       # sum_l n_l W_l I_l
        Kv = (w * t * I) @ mu                     # sum_l (u.n_l) n_l W_l I_l
        bracket = u @ Hvec - (uu * J + u @ Kv) / C
        rhsT = (-8 * np.pi * P * sa * bracket
                - P * C * (1 - uu / C ** 2) * sa * (T ** 4 - FOUR_PI * J))
        GT = cv * (T - Tn) - dt * rhsT
        return np.concatenate([G, [GT]])

    def jacobian(x):
        I, T = x[:N], x[N]
        Jm = np.zeros((N + 1, N + 1))
        Jm[:N, :N] = np.diag(1 + dt * C * sa - dt * t * sa)
        Jm[:N, :N] += dt * (sa * uu / C * w + sa / C * w * t * t)[None, :]
        Jm[:N, N] = -dt * (C * sa + 3 * t * sa) * T ** 3 / np.pi
        Jm[N, :N] = -dt * (-8 * np.pi * P * sa * (w * t - (uu * w + w * t * t) / C)
                           + P * C * (1 - uu / C ** 2) * sa * FOUR_PI * w)
        Jm[N, N] = cv + dt * P * C * (1 - uu / C ** 2) * sa * 4 * T ** 3
        return Jm

    prev = np.inf
    for it in range(1, maxit + 1):
        dx = np.linalg.solve(jacobian(x), -residual(x))
        x = x + dx
        step = max(abs(dx[N]) / abs(x[N]), np.max(np.abs(dx[:N])) / np.max(np.abs(x[:N])))
        if step <= tol:
            return x[:N], x[N], it
        # dense LU of a stiff Jacobian can stall at its rounding floor: stop
        # once the update no longer shrinks below that floor
        if step < 1e-11 and step >= prev:
            return x[:N], x[N], it
        prev = step
    raise RuntimeError("dense absorption Newton did not converge")


def scattering_matrix(mu, w, C, dt, ss, u):
    mu = np.asarray(mu, float)
    w = np.asarray(w, float)
    u = np.asarray(u, float)
    t = mu @ u
    uu = float(u @ u)
    a = (1 + dt * C * ss - dt * ss * t) / w
    b = -dt * C * ss + 2 * dt * ss * t - dt * ss * uu / C - dt * ss / C * t * t
    c = -3 * dt * t * ss
    N = len(w)
    M = np.empty((N, N))
    for m in range(N):
        for l in range(N):
            M[m, l] = b[l] + c[m] + (a[m] if m == l else 0.0)
    return M


def scattering_dense(mu, w, C, dt, ss, u, r):
    y = np.linalg.solve(scattering_matrix(mu, w, C, dt, ss, u), np.asarray(r, float))
    return y / np.asarray(w, float)


def _vl(a, b):
    ab = a * b
    with np.errstate(divide="ignore", invalid="ignore"):
        return np.where(ab > 0, 2 * ab / np.where(ab > 0, a + b, 1.0), 0.0)


def transport_periodic(shape, dx, mu, C, dt, I, J, v, sa, ss):
    """Delta F on a fully periodic grid (shape = (nz, ny, nx) active axes
    given by len(dx)), computed with array rolls.  I is (nang, nz, ny, nx),
    J, sa, ss are (nz, ny, nx), v is (3, nz, ny, nx)."""
    mu = np.asarray(mu, float)
    nang = mu.shape[0]
    ndim = len(dx)
    sig = sa + ss
    dF = np.zeros_like(I)
    for d in range(ndim):
        ax = 2 - d                      # array axis of physical axis d
        dl = dx[d]

        def sh(a, k, axis=ax):          # value at index i+k
            return np.roll(a, -k, axis=axis)

        # interface i-1/2 lies between cells i-1 and i
        sf = 0.5 * (sh(sig, -1) + sig)
        s = 10 * dl * sf
        tau = s * s
        with np.errstate(divide="ignore", invalid="ignore"):
            alpha = np.where(tau > 0, np.sqrt(-np.expm1(-tau) / np.where(tau > 0, tau, 1)), 1.0)
        uf = 0.5 * (sh(v[d], -1) + v[d])
        nuv = np.abs(uf) * dt / dl
        for m in range(nang):
            md = mu[m, d]
            IV = 3 * (mu[m, 0] * v[0] + mu[m, 1] * v[1] + mu[m, 2] * v[2]) * J
            It = I[m] - IV / C
            if md != 0:
                nu = C * abs(md) * dt / dl
                if md > 0:
                    up = sh(It, -1) + 0.5 * (1 - nu) * _vl(sh(It, -1) - sh(It, -2), It - sh(It, -1))
                else:
                    up = It + 0.5 * (1 - nu) * _vl(It - sh(It, 1), sh(It, -1) - It)
                cen = 0.5 * (sh(It, -1) + It)
                phi = C * md * (alpha * up + (1 - alpha) * cen)
            else:
                phi = np.zeros_like(It)
            ivp = sh(IV, -1) + 0.5 * (1 - nuv) * _vl(sh(IV, -1) - sh(IV, -2), IV - sh(IV, -1))
            ivm = IV + 0.5 * (1 - nuv) * _vl(IV - sh(IV, 1), sh(IV, -1) - IV)
            ivc = 0.5 * (sh(IV, -1) + IV)
            iv = np.where(uf > 0, ivp, np.where(uf < 0, ivm, ivc))
            flux = phi + md * iv             # flux through face i-1/2
            dF[m] -= dt * (sh(flux, 1) - flux) / dl
    return dF
