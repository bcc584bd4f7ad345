"""Oracle pin for the two-beam shadow problem (Section 5.8): with T held
fixed, no scattering and no flow, the steady state in every direction is the
formal solution of the transfer equation along straight rays
(``tests/rays.py``), which the discrete scheme approaches as the grid is
refined.  On cells where neither beam's ray passes near the cloud, the
oracle's steady E_r matches the ray solution to a few per cent on 32 x 16
cells and to better than half that error on 64 x 32 cells (second-order
transport, first-order near the kink where the beams from two faces meet);
behind the cloud, where both beam rays cross its opaque core, E_r falls to
under a tenth of its value in the lit region."""
import numpy as np
import pytest

import workloads as W
from rays import classify, ray_energy

FOUR_PI = 4.0 * np.pi


def _oracle_steady(nx, nsteps):
    import oracle
    wl = W.shadow2d(nx=nx, ny=nx // 2, nsteps=nsteps)
    ref = oracle.State(oracle.Problem(wl, estimate_v=False)).step(nsteps=nsteps)
    return wl, ref


def test_shadow2d_oracle_converges_to_ray_solution():
    errs = {}
    for nx, nsteps in ((32, 150), (64, 300)):   # > 1.5 light-crossing times
        wl, ref = _oracle_steady(nx, nsteps)
        lit, umbra = classify(wl)
        cells = np.where(lit)[0]
        cells = cells[:: max(1, len(cells) // 60)]
        Ea = ray_energy(wl, cells)
        errs[nx] = float(np.max(np.abs(ref.E[cells] - Ea) / Ea))
        print(f"shadow2d {nx}x{nx // 2}: lit cells {lit.sum()}, max rel error vs rays "
              f"{errs[nx]:.4f}; umbra cells {umbra.sum()}, E_umbra max "
              f"{ref.E[umbra].max() if umbra.any() else float('nan'):.3f}, "
              f"E_lit median {np.median(ref.E[lit]):.3f}", flush=True)
        if nx == 64:
            assert umbra.sum() > 0
            assert ref.E[umbra].max() < 0.1 * np.median(ref.E[lit])
    assert errs[32] < 0.06 and errs[64] < 0.025
    assert errs[64] < 0.6 * errs[32]


def test_shadow2d_beam_tables():
    """The beams enter where Section 5.8 puts them, at +-14 degrees."""
    wl = W.shadow2d(nx=32, ny=16)
    mu = np.asarray(wl.quad[1])
    up, down = wl.meta["beams"]
    assert np.degrees(np.arctan2(mu[up, 1], mu[up, 0])) == pytest.approx(14.0, abs=1e-9)
    assert np.degrees(np.arctan2(mu[down, 1], mu[down, 0])) == pytest.approx(-14.0, abs=1e-9)
    g = wl.ghost(mu)
    bg = 1.0 / FOUR_PI
    assert g[(0, 0)][up] == g[(0, 0)][down] == 103.13
    assert g[(1, 0)][up] == 103.13 and g[(1, 0)][down] == bg
    assert g[(1, 1)][down] == 103.13 and g[(1, 1)][up] == bg
    assert np.sum(np.asarray(wl.quad[2])) == pytest.approx(1.0, abs=1e-15)
