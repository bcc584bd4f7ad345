"""Two-dimensional beam problems of the paper's Section 5.

* ``shadow2d``: the shadow test (Section 5.8).  Box (-0.5, 0.5) x (-0.3, 0.3)
  at 512 x 256 cells, C = 10; background rho0 = 1, T0 = 1; inside the
  ellipse r = x^2/a^2 + y^2/b^2 (a = 0.1, b = 0.06) the density rises as
  rho0 + (rho1 - rho0)/(1 + exp(10 (r - 1))) with rho1 = 10 rho0; T = 1/rho
  and sigma_a = T^-3.5 rho^2, sigma_s = 0.  Beams of intensity 103.13 enter
  through the left face at +14 and -14 degrees to the x axis, through the
  bottom face at +14 degrees and through the top face at -14 degrees; the
  right face copies the last active cells.  The flow is not evolved.

Readings (the paper leaves them open): the directions are an in-plane set
of 90 equally weighted directions 4 degrees apart, which holds +-14 degrees
exactly; the gas temperature, and with it sigma_a, keeps its initial value
(a heat capacity so large that the temperature step leaves T unchanged),
and the velocity estimate is off (v = 0 throughout), so the steady state is
that of pure absorption and emission along each direction; the faces with
beams give the background equilibrium intensity 1/(4 pi) to every other
incoming direction.
"""
from __future__ import annotations

import math

import numpy as np

from .configs import BC_COPY, BC_FIXED, BC_PERIODIC, FOUR_PI, Workload, _cell_centres

HEAT_CAPACITY_R = 1e30
BEAM_INTENSITY = 103.13


def plane_directions(nphi: int = 90, phi0_deg: float = 2.0):
    """Directions in the x-y plane at phi0 + j 360/nphi degrees, equal
    weights summing to one: (mu (nphi, 3), w (nphi,))."""
    phi = np.radians(phi0_deg + np.arange(nphi) * (360.0 / nphi))
    mu = np.stack([np.cos(phi), np.sin(phi), np.zeros(nphi)], axis=1)
    return mu, np.full(nphi, 1.0 / nphi)


def direction_at(mu, deg: float) -> int:
    """Index of the direction of the table closest to deg degrees from +x
    in the x-y plane."""
    mu = np.asarray(mu)
    ang = np.degrees(np.arctan2(mu[:, 1], mu[:, 0]))
    diff = (ang - deg + 180.0) % 360.0 - 180.0
    return int(np.argmin(np.abs(diff)))


def shadow_density(x, y, a: float = 0.1, b: float = 0.06, rho0: float = 1.0,
                   rho1: float = 10.0):
    """Density of the shadow test at (x, y) (any array shape)."""
    r = (np.asarray(x) / a) ** 2 + (np.asarray(y) / b) ** 2
    with np.errstate(over="ignore"):
        return rho0 + (rho1 - rho0) / (1.0 + np.exp(10.0 * (r - 1.0)))


def shadow2d(nx: int = 512, ny: int = 256, nphi: int = 90, nsteps: int = 3000,
             C: float = 10.0, courant: float = 0.4, precision: str = "fp64",
             beam: float = BEAM_INTENSITY) -> Workload:
    n = (nx, ny, 1)
    dx = (1.0 / nx, 0.6 / ny, 1.0)
    X, Y, _ = _cell_centres(n, dx, origin=(-0.5, -0.3, 0.0))
    rho = shadow_density(X, Y)
    T = 1.0 / rho
    nc = nx * ny
    mu, w = plane_directions(nphi)
    up, down = direction_at(mu, 14.0), direction_at(mu, -14.0)
    bc = ((BC_FIXED, BC_COPY), (BC_FIXED, BC_FIXED), (BC_PERIODIC, BC_PERIODIC))
    wl = Workload(name=f"shadow2d-{nx}x{ny}-{nphi}dir", n=n, ndim=2, dx=dx, bc=bc,
                  quad=("table", mu, w), C=C, P=1.0, R=HEAT_CAPACITY_R, courant=courant,
                  nsteps=nsteps, precision=precision, rho=rho, T=T, v=np.zeros((3, nc)),
                  sigma_a=T ** -3.5 * rho ** 2, sigma_s=np.zeros(nc))
    wl.init = lambda m, T=T: np.broadcast_to(T ** 4 / FOUR_PI,
                                             (np.asarray(m).shape[0], nc)).copy()

    def ghost(m, up=up, down=down, beam=beam):
        bg = np.full(np.asarray(m).shape[0], 1.0 / FOUR_PI)
        left, bottom, top = bg.copy(), bg.copy(), bg.copy()
        left[[up, down]] = beam
        bottom[up] = beam
        top[down] = beam
        return {(0, 0): left, (1, 0): bottom, (1, 1): top}
    wl.ghost = ghost
    wl.meta.update(beams=(up, down), beam=beam, box=((-0.5, 0.5), (-0.3, 0.3)),
                   background=1.0 / FOUR_PI, estimate_v=False,
                   crossing_time=math.hypot(1.0, 0.6) / C)
    return wl
