"""Oracle pins for the crossing beams in vacuum (Section 5.4), at 16 x 64,
32 x 128 and 64 x 256 cells, once the beams have crossed the box:

* with no opacity the steady state conserves the flux: on every row the
  flux 4 pi sum_m w_m mu_y I_m dx equals the flux injected through the
  bottom face, to the discretisation error, which falls with resolution;
* each beam's centroid follows its 45-degree line through the periodic
  wraps and the crossings (the beams pass through each other);
* the beams widen only by numerical diffusion, whose variance growth over a
  unit height halves when the cells halve (first order at the beam edges);
* the other directions stay exactly zero and T exactly 1."""
import numpy as np

import workloads as W
from rays import beam_stats
from golden_values import golden


def _run(nx):
    import oracle
    nsteps = 19 * nx  # dt = 0.4/nx: 1.34 light-crossing times of the box height
    wl = W.crossing_beams(nx=nx, ny=4 * nx, nsteps=nsteps)
    ref = oracle.State(oracle.Problem(wl, estimate_v=False)).step(nsteps=nsteps)
    assert nsteps * wl.dt > wl.meta["crossing_time"]
    return wl, ref


def test_crossing_beams_oracle_pins():
    dev, cen, growth = {}, {}, {}
    for nx in (16, 32, 64):
        wl, ref = _run(nx)
        st = beam_stats(wl, ref.I)
        dev[nx] = float(np.abs(st["row_flux"] / st["injected"] - 1.0).max())
        cen[nx] = max(float(np.abs(b["centroid_error"]).max()) / wl.dx[0] for b in st["beams"])
        j = int(1.0 / wl.dx[1])  # the row at unit height
        growth[nx] = [float(b["var"][j] - b["var"][0]) for b in st["beams"]]
        print(f"crossing beams {nx}x{4 * nx}: row flux deviation {dev[nx]:.4f}, centroid error "
              f"{cen[nx]:.2f} cells, variance growth at y = 1 {growth[nx]}", flush=True)
        R, L = wl.meta["beams"]
        others = np.delete(np.asarray(ref.I), [R, L], axis=0)
        assert np.all(others == 0.0) and np.all(ref.T == 1.0)
    assert dev[32] < 0.015 and dev[64] < dev[32] < dev[16] < 0.03
    assert cen[16] < 1.5 and cen[32] < 0.75 and cen[64] < 0.75
    for a, b in ((16, 32), (32, 64)):
        for ga, gb in zip(growth[a], growth[b]):
            assert 0.4 < gb / ga < 0.6


def test_crossing_beam_windows():
    s = golden("sec5_4_crossing_beams.json")
    full = W.crossing_beams()
    assert [full.n[0], full.n[1]] == s["resolutions"][0]
    assert (full.n[0] * full.dx[0], full.n[1] * full.dx[1]) == tuple(s["box"])
    assert full.bc[0] == (W.BC_PERIODIC, W.BC_PERIODIC) and np.all(full.sigma_a == 0.0)
    assert np.all(full.sigma_s == s["sigma_s"])
    wl = W.crossing_beams(nx=32, ny=128)
    mu = np.asarray(wl.quad[1])
    R, L = wl.meta["beams"]
    assert [np.degrees(np.arctan2(mu[m, 1], mu[m, 0])) for m in (R, L)] == \
        s["beam_angles_deg_from_plus_x"]
    g = wl.ghost_face(mu)[(1, 0)]
    assert g.shape == (4, 32)
    assert g[R].sum() == 4 and g[L].sum() == 4           # 1/8 of the face each
    assert np.all(g[R, 6:10] == 1.0) and np.all(g[L, 22:26] == 1.0)
    assert np.all(np.delete(g, [R, L], axis=0) == 0.0)
