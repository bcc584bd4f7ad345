"""The non-LTE atmosphere (paper Section 5.3) as a 1D slab along x.

The paper's box is (-0.5, 0.5)^2 x (-10, 10) at 16 x 16 x 1280 cells with
periodic x and y; the fields depend on the vertical coordinate only, so one
column is the same problem.  Density 1e-3 exp(10 - z), sigma_a = eps rho,
sigma_s = (1 - eps) rho, T = 1 held fixed (a heat capacity large enough that
the temperature step leaves it at 1), v = 0, one direction per octant (the
level-symmetric set of order 2), I = 1/(4 pi) initially; the lower face
copies all directions from the last cell, the upper face copies outgoing
directions and gives zero to incoming ones.  Optical depth from the top:
tau(z) = 1e-3 (e^{10 - z} - 1).
"""
from __future__ import annotations

import numpy as np

from .configs import BC_COPY, BC_VACUUM, small_case

HEAT_CAPACITY_R = 1e30


def atmosphere(eps: float, ncell: int = 1280, C: float = 1.0, courant: float = 0.4):
    wl = small_case(1, (ncell,), ("ls", 2), seed=1, courant=courant, C=C, P=1.0, kappa_a=0.0,
                    kappa_s=0.0, vscale=0.0, bc=((BC_COPY, BC_VACUUM), (0, 0), (0, 0)))
    dz = 20.0 / ncell
    wl.dx = (dz, 1.0, 1.0)
    z = -10.0 + (np.arange(ncell) + 0.5) * dz
    rho = 1e-3 * np.exp(10.0 - z)
    wl.rho[:] = rho
    wl.T[:] = 1.0
    wl.v[:] = 0.0
    wl.sigma_a[:] = eps * rho
    wl.sigma_s[:] = (1.0 - eps) * rho
    wl.R = HEAT_CAPACITY_R
    wl.init = lambda mu, nc=ncell: np.full((np.asarray(mu).shape[0], nc), 1.0 / (4.0 * np.pi))
    wl.name = f"atmosphere-eps{eps:g}"
    wl.meta.update(eps=eps, tau=1e-3 * (np.exp(10.0 - z) - 1.0))
    return wl
