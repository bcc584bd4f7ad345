"""Two-dimensional beam problems of the paper's Section 5.

* ``shadow2d``: the shadow test (Section 5.8).  Box (-0.5, 0.5) x (-0.3, 0.3)
  at 512 x 256 cells, C = 10; background rho0 = 1, T0 = 1; inside the
  ellipse r = x^2/a^2 + y^2/b^2 (a = 0.1, b = 0.06) the density rises as
  rho0 + (rho1 - rho0)/(1 + exp(10 (r - 1))) with rho1 = 10 rho0; T = 1/rho
  and sigma_a = T^-3.5 rho^2, sigma_s = 0.  Beams of intensity 103.13 enter
  through the left face at +14 and -14 degrees to the x axis, through the
  bottom face at +14 degrees and through the top face at -14 degrees; the
  right face copies the last active cells.  The flow is not evolved.

* ``crossing_beams``: two beams crossing vacuum (Section 5.4).  Box
  L_x = 1, L_y = 4 at 128 x 512 cells (the paper also runs 256 x 1024),
  periodic along x, zero absorption and scattering; beams enter through the
  bottom face at 45 degrees to the +x and to the -x axis, wrap around
  through the periodic x faces, cross and leave through the top.

Readings of the shadow test (the paper leaves them open): the directions are an in-plane set
of 90 equally weighted directions 4 degrees apart, which holds +-14 degrees
exactly; the gas temperature, and with it sigma_a, keeps its initial value
(a heat capacity so large that the temperature step leaves T unchanged),
and the velocity estimate is off (v = 0 throughout), so the steady state is
that of pure absorption and emission along each direction; the faces with
beams give the background equilibrium intensity 1/(4 pi) to every other
incoming direction.

Readings of the crossing beams: each beam enters through a window of width
1/8 of the bottom face, the +x beam centred at x = 1/4 and the -x beam at
x = 3/4, so that they cross inside the box every 1/2 in height; unit beam
intensity, zero elsewhere on the face and zero initial intensity; C = 1;
the directions are the four in-plane ones at 45 + 90 k degrees; the top face
is a vacuum face (outgoing copied, incoming zero), through which the beams
leave.
"""
from __future__ import annotations

import math

import numpy as np

from .configs import (BC_COPY, BC_FIXED, BC_PERIODIC, BC_VACUUM, FOUR_PI, Workload,
                      _cell_centres)

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


def crossing_beams(nx: int = 128, ny: int = 512, nsteps: int = 2400, C: float = 1.0,
                   courant: float = 0.4, precision: str = "fp64", width: float = 0.125,
                   centres=(0.25, 0.75), beam: float = 1.0) -> Workload:
    n = (nx, ny, 1)
    dx = (1.0 / nx, 4.0 / ny, 1.0)
    nc = nx * ny
    mu, w = plane_directions(4, 45.0)
    right, left = direction_at(mu, 45.0), direction_at(mu, 135.0)
    bc = ((BC_PERIODIC, BC_PERIODIC), (BC_FIXED, BC_VACUUM), (BC_PERIODIC, BC_PERIODIC))
    wl = Workload(name=f"crossing-beams-{nx}x{ny}", n=n, ndim=2, dx=dx, bc=bc,
                  quad=("table", mu, w), C=C, P=1.0, courant=courant, nsteps=nsteps,
                  precision=precision, rho=np.ones(nc), T=np.ones(nc), v=np.zeros((3, nc)),
                  sigma_a=np.zeros(nc), sigma_s=np.zeros(nc))
    wl.init = lambda m: np.zeros((np.asarray(m).shape[0], nc))
    xs = (np.arange(nx) + 0.5) / nx

    def window(c):
        dist = np.abs((xs - c + 0.5) % 1.0 - 0.5)
        return (dist < 0.5 * width).astype(np.float64)

    def ghost(m):
        return {(1, 0): np.zeros(np.asarray(m).shape[0])}

    def ghost_face(m, right=right, left=left):
        g = np.zeros((np.asarray(m).shape[0], nx))
        g[right] = beam * window(centres[0])
        g[left] = beam * window(centres[1])
        return {(1, 0): g}
    wl.ghost = ghost
    wl.ghost_face = ghost_face
    wl.meta.update(beams=(right, left), centres=centres, width=width, beam=beam,
                   window_cells=(window(centres[0]).sum(), window(centres[1]).sum()),
                   crossing_time=4.0 * math.sqrt(2.0) / C)
    return wl
