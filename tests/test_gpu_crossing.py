"""Crossing beams in vacuum (Section 5.4) on the GPU, with beams entering
through part of the bottom face (``rt_set_fixed_bc_face``).

* A 32 x 128 copy matches the oracle after 300 steps: FP64 within 1e-12,
  FP32-mixed within 1e-5.
* At the paper's 128 x 512 and 256 x 1024 cells, once the beams have
  crossed the box: every row carries the injected flux (within 1%: the
  cell-centred row flux differs from the conserved interface flux by the
  reconstruction slopes), each beam's centroid follows its 45-degree line
  through the periodic wraps and the crossings (within a cell), the beams
  stay apart between crossings (E_r midway between them under 5% of the
  peak, the tails of beams widened by numerical diffusion: merged beams
  would peak there), and the numerical widening of the beams halves with
  the cell size."""
import numpy as np
import pytest

import workloads as W
from rays import beam_stats

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "mixed": 1e-5}


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_crossing_copy_matches_oracle(precision):
    import oracle

    from paper_1403_6126_amd.solver import Solver
    wl = W.crossing_beams(nx=32, ny=128, nsteps=300, precision=precision)
    print(f"case {wl.name} {precision}: 300 steps against the oracle", flush=True)
    ref = oracle.State(oracle.Problem(wl, estimate_v=False)).step(nsteps=300)
    s = Solver(wl, precision=precision, estimate_v=False)
    s.step(300)
    st = s.state()
    status = s.status()
    s.close()
    assert status == 0
    errs = {k: float(np.abs(st[k] - r).max() / np.abs(r).max())
            for k, r in (("I", ref.I), ("E", ref.E), ("F", ref.F))}
    print("   errors", errs, flush=True)
    assert max(errs.values()) <= TOL[precision], errs


def test_crossing_full_size():
    from paper_1403_6126_amd.solver import Solver
    growth = {}
    for nx in (128, 256):
        wl = W.crossing_beams(nx=nx, ny=4 * nx, nsteps=19 * nx)
        print(f"case {wl.name}: {wl.nsteps} steps, FP64", flush=True)
        s = Solver(wl, estimate_v=False)
        s.step(wl.nsteps)
        st = s.state()
        status = s.status()
        s.close()
        assert status == 0
        assert wl.nsteps * wl.dt > wl.meta["crossing_time"]
        b = beam_stats(wl, st["I"])
        dev = float(np.abs(b["row_flux"] / b["injected"] - 1.0).max())
        cen = max(float(np.abs(x["centroid_error"]).max()) for x in b["beams"]) / wl.dx[0]
        j = int(1.0 / wl.dx[1])
        growth[nx] = [float(x["var"][j] - x["var"][0]) for x in b["beams"]]
        # at unit height the +x beam is back at x = 1/4 and the -x beam at 3/4
        E = st["E"].reshape(wl.n[1], wl.n[0])[j]
        mid = E[[0, nx // 2 - 1, nx // 2, nx - 1]].max()
        print(f"   row flux deviation {dev:.5f}, centroid error {cen:.3f} cells, variance "
              f"growth at y = 1 {growth[nx]}, E_r midway / peak {mid / E.max():.2e}", flush=True)
        assert dev <= 1e-2 and cen <= 1.0 and mid < 0.05 * E.max()
    for a, b in zip(growth[128], growth[256]):
        assert 0.4 < b / a < 0.6


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_uniform_face_table_equals_angle_table(precision):
    """A position-dependent table that is the same on every face cell gives
    the step of the per-angle table bit for bit (both kernels read the same
    value for every ghost), on fixed faces of all six sides of a 3D grid
    and of the thread-per-cell kernel (more than 320 directions); a later
    rt_set_fixed_bc puts the face back on its angle table."""
    from paper_1403_6126_amd import rt
    from paper_1403_6126_amd.solver import Solver
    fixed = ((rt.RT_BC_FIXED, rt.RT_BC_FIXED),) * 3
    cases = [W.small_case(3, (12, 10, 9), ("ls", 8), seed=81, bc=fixed, ghost_seed=82,
                          precision=precision),
             W.small_case(1, (40,), ("gl", 330), seed=83, bc=fixed, ghost_seed=84,
                          precision=precision)]
    for wl in cases:
        ref = Solver(wl, precision=precision)
        ref.step(4)
        a = ref.state()
        tables = wl.ghost(np.asarray(ref.mu))
        face = {}
        for (axis, side), tab in tables.items():
            if axis < wl.ndim:
                nface = wl.ncell // wl.n[axis]
                face[(axis, side)] = np.repeat(np.asarray(tab)[:, None], nface, axis=1)
        wl.ghost_face = lambda mu, face=face: face
        s = Solver(wl, precision=precision)
        s.step(4)
        b = s.state()
        print(f"case {wl.name} {precision}: uniform face tables vs angle tables", flush=True)
        for k in ("I", "T", "E", "F"):
            assert np.array_equal(a[k], b[k]), k
        # back to the angle tables, with a different table on one face in both
        # runs: the two continue to agree
        for (axis, side), tab in tables.items():
            if axis < wl.ndim:
                t2 = np.asarray(tab) * (1.5 if (axis, side) == (0, 0) else 1.0)
                rt.rt_set_fixed_bc(s.ctx, axis, side, t2)
                rt.rt_set_fixed_bc(ref.ctx, axis, side, t2)
        ref.step(3)
        s.step(3)
        a, b = ref.state(), s.state()
        ref.close()
        s.close()
        for k in ("I", "T", "E", "F"):
            assert np.array_equal(a[k], b[k]), k


def test_face_table_arguments():
    from paper_1403_6126_amd import rt
    from paper_1403_6126_amd.solver import Solver
    bc = ((rt.RT_BC_FIXED, rt.RT_BC_VACUUM), (rt.RT_BC_PERIODIC, rt.RT_BC_PERIODIC),
          (rt.RT_BC_PERIODIC, rt.RT_BC_PERIODIC))
    wl = W.small_case(2, (8, 6), ("ls", 4), seed=85, bc=bc)
    s = Solver(wl)
    tab = np.zeros((len(s.mu), wl.ncell // wl.n[0]))
    rt.rt_set_fixed_bc_face(s.ctx, 0, 0, tab)               # fixed face: accepted
    for axis, side in ((0, 1), (1, 0), (2, 0), (-1, 0), (0, 2)):
        with pytest.raises(rt.RTError) as e:
            rt.rt_set_fixed_bc_face(s.ctx, axis, side, tab)  # not fixed, inactive or bad face
        assert e.value.status == rt.RT_EINVAL
    s.close()
