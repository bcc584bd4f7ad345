"""Workload definitions: grids, fields, initial intensities, boundary tables.

Every random draw uses ``numpy.random.Generator(PCG64(seed))`` and arrays are
drawn in C order of ``(nz, ny, nx)`` (x fastest), in the order rho, T, v.
"Lognormal(s)" means ``exp(s*z)`` with ``z ~ N(0, 1)`` (median 1).

Code units follow the paper's dimensionless form (Crat = c, Prat; the
equilibrium intensity is T^4/4pi).  Unless a workload says otherwise:
C = 1, P = 1, gamma = 5/3, R_ideal = 1, box length 1 per axis, dx = 1/n.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional, Tuple

import numpy as np

BC_PERIODIC, BC_FIXED, BC_COPY, BC_VACUUM = 0, 1, 2, 3

FOUR_PI = 4.0 * math.pi


def lognormal(rng: np.random.Generator, s: float, size) -> np.ndarray:
    return np.exp(s * rng.standard_normal(size))


@dataclass
class Workload:
    """One radiative-transfer problem instance (inputs only)."""
    name: str
    n: Tuple[int, int, int]                 # (nx, ny, nz); unused axes are 1
    ndim: int
    dx: Tuple[float, float, float]
    bc: Tuple[Tuple[int, int], ...]         # bc[axis][side], side 0 = low
    quad: Tuple                              # ("gl", n) | ("ls", order) | ("table", mu, w)
    C: float = 1.0
    P: float = 1.0
    gamma: float = 5.0 / 3.0
    R: float = 1.0
    courant: float = 0.5                     # dt = courant * min(dx) / C
    nsteps: int = 1
    precision: str = "fp64"                  # "fp64" | "mixed"
    rho: Optional[np.ndarray] = None
    T: Optional[np.ndarray] = None
    v: Optional[np.ndarray] = None           # (3, ncell)
    sigma_a: Optional[np.ndarray] = None
    sigma_s: Optional[np.ndarray] = None
    # initial intensity from the angle table: I0(mu (nang,3)) -> (nang, ncell)
    init: Optional[Callable[[np.ndarray], np.ndarray]] = None
    # fixed-boundary tables from the angle table: {(axis, side): (nang,)}
    ghost: Optional[Callable[[np.ndarray], Dict[Tuple[int, int], np.ndarray]]] = None
    # position-dependent fixed-boundary tables: {(axis, side): (nang, nface)},
    # face cells ordered by the two other axes, lower axis fastest
    ghost_face: Optional[Callable[[np.ndarray], Dict[Tuple[int, int], np.ndarray]]] = None
    meta: Dict = field(default_factory=dict)

    @property
    def ncell(self) -> int:
        return self.n[0] * self.n[1] * self.n[2]

    @property
    def dt(self) -> float:
        active = [self.dx[d] for d in range(self.ndim)]
        return self.courant * min(active) / self.C

    @property
    def cell_volume(self) -> float:
        vol = 1.0
        for d in range(self.ndim):
            vol *= self.dx[d]
        return vol


def equilibrium_intensity(T: np.ndarray, nang: int, xp=np) -> np.ndarray:
    """I_m = T^4 / 4pi for every angle: the initial state of most workloads."""
    base = T ** 4 / FOUR_PI
    if xp is np:
        return np.broadcast_to(base, (nang, base.shape[0])).copy()
    return base.unsqueeze(0).expand(nang, base.shape[0])


def moment_intensity(mu, E, F, xp=np):
    """I_m = (E + 3 n_m . F) / 4pi, the intensity with given E and F whose
    pressure is isotropic (first-order angular expansion)."""
    if xp is np:
        mu = np.asarray(mu)
        return (E[None, :] + 3.0 * (mu @ F)) / FOUR_PI
    return (E.unsqueeze(0) + 3.0 * (mu @ F)) / FOUR_PI


def _cell_centres(n, dx, origin=(0.0, 0.0, 0.0)):
    xs = [origin[d] + (np.arange(n[d]) + 0.5) * dx[d] for d in range(3)]
    Z, Y, X = np.meshgrid(xs[2], xs[1], xs[0], indexing="ij")
    return X.ravel(), Y.ravel(), Z.ravel()


def _grid(ndim: int, nper: Tuple[int, ...], box=(1.0, 1.0, 1.0)):
    n = [1, 1, 1]
    dx = [1.0, 1.0, 1.0]
    for d in range(ndim):
        n[d] = int(nper[d])
        dx[d] = box[d] / n[d]
    return tuple(n), tuple(dx)


def _periodic(ndim):
    return tuple((BC_PERIODIC, BC_PERIODIC) for _ in range(3))


# --------------------------------------------------------------------------
# Configuration 1: 1D periodic slab, 512 cells, 16 Gauss-Legendre directions.
# --------------------------------------------------------------------------
def config1(ncell: int = 512, seed: int = 1, nsteps: int = 100, nang: int = 16,
            precision: str = "fp64") -> Workload:
    n, dx = _grid(1, (ncell,))
    rng = np.random.Generator(np.random.PCG64(seed))
    rho = lognormal(rng, 0.5, ncell)
    T = lognormal(rng, 0.5, ncell)
    v = np.zeros((3, ncell))
    v[0] = rng.uniform(-0.01, 0.01, ncell)
    w = Workload(name="slab1d-512-gl16", n=n, ndim=1, dx=dx, bc=_periodic(1),
                 quad=("gl", nang), courant=0.5, nsteps=nsteps, precision=precision,
                 rho=rho, T=T, v=v, sigma_a=1.0 * rho, sigma_s=10.0 * rho)
    w.init = lambda mu, T=T: equilibrium_intensity(T, mu.shape[0])
    return w


# --------------------------------------------------------------------------
# Configuration 2: 3D periodic box, S8 level-symmetric (80 directions).
# --------------------------------------------------------------------------
def config2(nper: int = 128, seed: int = 2, nsteps: int = 50, order: int = 8,
            precision: str = "fp64", shape=None) -> Workload:
    shape = shape or (nper, nper, nper)
    n, dx = _grid(3, shape)
    nc = n[0] * n[1] * n[2]
    rng = np.random.Generator(np.random.PCG64(seed))
    rho = lognormal(rng, 1.0, nc)
    T = lognormal(rng, 0.3, nc)
    v = rng.normal(0.0, 0.02, (3, nc))
    w = Workload(name=f"box3d-{shape[0]}x{shape[1]}x{shape[2]}-s{order}", n=n, ndim=3,
                 dx=dx, bc=_periodic(3), quad=("ls", order), courant=0.4,
                 nsteps=nsteps, precision=precision, rho=rho, T=T, v=v,
                 sigma_a=0.1 * rho, sigma_s=1.0 * rho)
    w.init = lambda mu, T=T: equilibrium_intensity(T, mu.shape[0])
    return w


# --------------------------------------------------------------------------
# Configuration 3: shadow geometry (optically thin background, dense clump,
# collimated beam injected through the -x face).
# --------------------------------------------------------------------------
def config3(nper: int = 256, seed: int = 3, nsteps: int = 50, order: int = 8,
            precision: str = "mixed", beam: float = 103.13) -> Workload:
    n, dx = _grid(3, (nper, nper, nper))
    rng = np.random.Generator(np.random.PCG64(seed))
    centre = np.array([0.08, 0.5, 0.5]) + rng.uniform(-0.01, 0.01, 3)
    axes = np.array([0.04, 0.08, 0.08]) * (1.0 + rng.uniform(-0.1, 0.1, 3))
    X, Y, Z = _cell_centres(n, dx)
    r = ((X - centre[0]) / axes[0]) ** 2 + ((Y - centre[1]) / axes[1]) ** 2 \
        + ((Z - centre[2]) / axes[2]) ** 2
    rho0, rho1 = 1.0, 1.0e3
    # logistic edge of the clump; exp overflow far outside is harmless (-> rho0)
    with np.errstate(over="ignore"):
        rho = rho0 + (rho1 - rho0) / (1.0 + np.exp(10.0 * (r - 1.0)))
    T = 1.0 / rho
    nc = rho.size
    kappa_a = 0.256
    bc = tuple((BC_FIXED, BC_FIXED) for _ in range(3))
    w = Workload(name=f"shadow3d-{nper}-s{order}", n=n, ndim=3, dx=dx, bc=bc,
                 quad=("ls", order), courant=0.4, nsteps=nsteps, precision=precision,
                 rho=rho, T=T, v=np.zeros((3, nc)), sigma_a=kappa_a * rho,
                 sigma_s=np.zeros(nc))
    w.init = lambda mu, T=T: equilibrium_intensity(T, mu.shape[0])

    def ghost(mu, beam=beam):
        mu = np.asarray(mu)
        bg = np.full(mu.shape[0], 1.0 / FOUR_PI)
        tables = {(a, s): bg.copy() for a in range(3) for s in range(2)}
        cand = np.where((mu[:, 1] > 0) & (mu[:, 2] > 0))[0]
        mstar = cand[np.argmax(mu[cand, 0])]
        tables[(0, 0)][mstar] = beam
        return tables
    w.ghost = ghost
    w.meta.update(centre=centre, axes=axes)
    return w


# --------------------------------------------------------------------------
# Configuration 5: optically thick advective diffusion of a Gaussian pulse.
# --------------------------------------------------------------------------
def config5(shape=(512, 512, 256), width_cells: float = 32.0, nsteps: int = 100,
            order: int = 8, precision: str = "mixed", sigma_s: float = 1.0e3,
            vx: float = 0.03) -> Workload:
    dxx = 1.0 / 512.0
    n = tuple(int(s) for s in shape)
    dx = (dxx, dxx, dxx)
    nc = n[0] * n[1] * n[2]
    box = [n[d] * dx[d] for d in range(3)]
    C = 1.0
    wid = width_cells * dxx
    X, Y, Z = _cell_centres(n, dx)
    x0 = [0.5 * box[0], 0.5 * box[1], 0.5 * box[2]]
    g = np.exp(-((X - x0[0]) ** 2 + (Y - x0[1]) ** 2 + (Z - x0[2]) ** 2) / (2 * wid ** 2))
    E = 1.0 + g
    grad = np.stack([-(X - x0[0]) / wid ** 2 * g, -(Y - x0[1]) / wid ** 2 * g,
                     -(Z - x0[2]) / wid ** 2 * g])
    v = np.zeros((3, nc))
    v[0] = vx
    F = -grad / (3.0 * sigma_s) + 4.0 * v * E[None, :] / (3.0 * C)
    w = Workload(name=f"diffusion3d-{n[0]}x{n[1]}x{n[2]}-s{order}", n=n, ndim=3,
                 dx=dx, bc=_periodic(3), quad=("ls", order), C=C, courant=0.4,
                 nsteps=nsteps, precision=precision, rho=np.ones(nc), T=np.ones(nc),
                 v=v, sigma_a=np.zeros(nc), sigma_s=np.full(nc, sigma_s))
    w.init = lambda mu, E=E, F=F: moment_intensity(mu, E, F)
    w.meta.update(E0=E, F0=F, centre=x0, width=wid, diffusion=C / (3.0 * sigma_s))
    return w


# --------------------------------------------------------------------------
# Configuration 4: a stream of independent solves for the serving loop.
# --------------------------------------------------------------------------
LS_TOTALS = {24: 4, 48: 6, 80: 8, 120: 10, 168: 12, 224: 14, 288: 16}


def config4_requests(count: int = 2000, seed: int = 4, min_cells: int = 64,
                     max_cells: int = 128 ** 3, min_steps: int = 10,
                     max_steps: int = 200) -> List[Dict]:
    """Request descriptors (no arrays): arrival gaps are unit-rate exponential
    draws that the caller scales by 1/lambda."""
    rng = np.random.Generator(np.random.PCG64(seed))
    reqs = []
    for i in range(count):
        gap = rng.exponential(1.0)
        ncell = int(round(math.exp(rng.uniform(math.log(min_cells), math.log(max_cells)))))
        ndim = int(rng.integers(1, 4))
        if ndim == 1:
            shape = (ncell,)
            nang = int(rng.integers(8, 145)) * 2          # even, 16..288
            quad = ("gl", nang)
        else:
            side = max(2, int(round(ncell ** (1.0 / ndim))))
            shape = (side,) * ndim
            total = int(rng.choice(sorted(LS_TOTALS)))
            quad = ("ls", LS_TOTALS[total])
        nsteps = int(rng.integers(min_steps, max_steps + 1))
        reqs.append(dict(id=i, gap=gap, ndim=ndim, shape=shape, quad=quad,
                         nsteps=nsteps, seed=4_000_000 + i))
    return reqs


REQUEST_DX = 1.0 / 512


def request_workload(req: Dict, precision: str = "mixed") -> Workload:
    """Fields of one serving request: as configuration 1 (lognormal rho and T,
    sigma_a = rho, sigma_s = 10 rho, cells of size 1/512, so the optical
    depth per cell is that of configuration 1 whatever the grid) with every
    velocity component uniform in [-0.01, 0.01]."""
    ndim = req["ndim"]
    shape = tuple(req["shape"])
    n, dx = _grid(ndim, shape, box=tuple(s * REQUEST_DX for s in shape) + (1.0,) * (3 - ndim))
    nc = n[0] * n[1] * n[2]
    rng = np.random.Generator(np.random.PCG64(req["seed"]))
    rho = lognormal(rng, 0.5, nc)
    T = lognormal(rng, 0.5, nc)
    v = np.zeros((3, nc))
    ncomp = 1 if req["quad"][0] == "gl" else 3
    v[:ncomp] = rng.uniform(-0.01, 0.01, (ncomp, nc))
    # Courant number 0.5 along the fastest ray, as in configuration 1: the sum
    # over the axes of |n_d| C dt / dx is at most 0.5 (|n| = 1 gives
    # sum_d |n_d| <= sqrt(ndim)), the range in which the unsplit limited
    # transport keeps intensities non-negative.
    w = Workload(name=f"request-{req['id']}", n=n, ndim=ndim, dx=dx,
                 bc=_periodic(ndim), quad=req["quad"], courant=0.5 / math.sqrt(ndim),
                 nsteps=req["nsteps"], precision=precision, rho=rho, T=T, v=v,
                 sigma_a=rho.copy(), sigma_s=10.0 * rho)
    w.init = lambda mu, T=T: equilibrium_intensity(T, mu.shape[0])
    return w


# --------------------------------------------------------------------------
# Small cases for parity tests (several tiles plus a ragged tail).
# --------------------------------------------------------------------------
def small_case(ndim: int, shape, quad, seed: int = 11, nsteps: int = 3,
               courant: float = 0.4, kappa_a: float = 1.0, kappa_s: float = 1.0,
               vscale: float = 0.02, rho_s: float = 1.0, T_s: float = 0.3,
               bc=None, precision: str = "fp64", C: float = 1.0, P: float = 1.0,
               ghost_seed: Optional[int] = None) -> Workload:
    n, dx = _grid(ndim, shape)
    nc = n[0] * n[1] * n[2]
    rng = np.random.Generator(np.random.PCG64(seed))
    rho = lognormal(rng, rho_s, nc)
    T = lognormal(rng, T_s, nc)
    v = np.zeros((3, nc))
    v[:] = rng.normal(0.0, vscale, (3, nc))
    if ndim == 1 and quad[0] == "gl":
        v[1:] = 0.0
    bc = bc or _periodic(ndim)
    w = Workload(name=f"small{ndim}d-{'x'.join(map(str, shape))}", n=n, ndim=ndim,
                 dx=dx, bc=bc, quad=quad, C=C, P=P, courant=courant, nsteps=nsteps,
                 precision=precision, rho=rho, T=T, v=v, sigma_a=kappa_a * rho,
                 sigma_s=kappa_s * rho)
    w.init = lambda mu, T=T: equilibrium_intensity(T, mu.shape[0])
    if ghost_seed is not None:
        def ghost(mu, seed=ghost_seed):
            g = np.random.Generator(np.random.PCG64(seed))
            return {(a, s): g.uniform(0.0, 0.2, np.asarray(mu).shape[0])
                    for a in range(3) for s in range(2)}
        w.ghost = ghost
    return w
