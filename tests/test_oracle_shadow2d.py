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
from golden_values import golden

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


def test_shadow2d_setup_is_the_papers():
    """The workload is the printed setup of Section 5.8: box, resolution,
    Crat, cloud, and the beams where the paper puts them."""
    s = golden("sec5_8_shadow.json")
    wl = W.shadow2d()
    assert (wl.n[0], wl.n[1]) == tuple(s["resolution"]) and wl.C == s["Crat"]
    assert wl.meta["box"] == tuple(tuple(b) for b in s["box"])
    assert wl.dx[0] * wl.n[0] == pytest.approx(s["box"][0][1] - s["box"][0][0])
    assert wl.dx[1] * wl.n[1] == pytest.approx(s["box"][1][1] - s["box"][1][0])
    assert W.shadow_density(0.0, 0.0) == pytest.approx(
        s["rho0"] + (s["rho1_over_rho0"] - 1.0) * s["rho0"] / (1.0 + np.exp(-10.0)))
    assert W.shadow_density(s["ellipse_a"], 0.0) == pytest.approx(
        s["rho0"] + 0.5 * (s["rho1_over_rho0"] - 1.0) * s["rho0"])   # r = 1 on the ellipse
    assert W.shadow_density(0.0, s["ellipse_b"]) == pytest.approx(
        s["rho0"] + 0.5 * (s["rho1_over_rho0"] - 1.0) * s["rho0"])
    far = W.shadow_density(0.45, 0.25)
    assert far == pytest.approx(s["rho0"]) and wl.T.max() == pytest.approx(1.0 / s["rho0"])
    mu = np.asarray(wl.quad[1])
    up, down = wl.meta["beams"]
    ang = {"up": np.degrees(np.arctan2(mu[up, 1], mu[up, 0])),
           "down": np.degrees(np.arctan2(mu[down, 1], mu[down, 0]))}
    assert sorted(s["beam_angles_deg"]["left"]) == pytest.approx(sorted(ang.values()), abs=1e-9)
    assert s["beam_angles_deg"]["bottom"] == pytest.approx([ang["up"]], abs=1e-9)
    assert s["beam_angles_deg"]["top"] == pytest.approx([ang["down"]], abs=1e-9)
    g = wl.ghost(mu)
    bg = 1.0 / FOUR_PI
    beam = s["beam_intensity"]
    assert g[(0, 0)][up] == g[(0, 0)][down] == beam
    assert g[(1, 0)][up] == beam and g[(1, 0)][down] == bg
    assert g[(1, 1)][down] == beam and g[(1, 1)][up] == bg
    assert np.sum(np.asarray(wl.quad[2])) == pytest.approx(1.0, abs=1e-15)
