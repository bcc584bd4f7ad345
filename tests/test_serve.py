"""Serving runtime (include/rt_serve.h) on the GPU: results are the same
alone and in a mix (bit for bit), equal to the plain rt_step path, and
within the mixed-precision tolerance of the oracle; admission respects the
arena and slot limits."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

TOL_MIXED = 1e-5


def _mix():
    """Requests spanning packed (small, FP32) and chunked launches, 1D/2D/3D,
    10 to 288 directions, ragged tiles."""
    specs = [
        dict(ndim=1, shape=(64,), quad=("gl", 16), nsteps=7),
        dict(ndim=1, shape=(333,), quad=("gl", 288), nsteps=5),
        dict(ndim=2, shape=(9, 9), quad=("ls", 6), nsteps=6),
        dict(ndim=2, shape=(23, 23), quad=("ls", 12), nsteps=4),
        dict(ndim=3, shape=(4, 4, 4), quad=("ls", 4), nsteps=9),
        dict(ndim=3, shape=(7, 7, 7), quad=("ls", 16), nsteps=3),
        dict(ndim=3, shape=(19, 19, 19), quad=("ls", 8), nsteps=5),
        dict(ndim=2, shape=(71, 71), quad=("ls", 10), nsteps=4),
        dict(ndim=1, shape=(5000,), quad=("gl", 40), nsteps=8),
        dict(ndim=3, shape=(26, 26, 26), quad=("ls", 14), nsteps=2),
    ]
    wls = []
    for i, s in enumerate(specs):
        req = dict(id=i, seed=4_100_000 + i, **s)
        wls.append(W.request_workload(req, precision="mixed"))
    return wls


SERVER = dict(pool_bytes=4 << 30, max_active=64, packed_cells=2048, chunk_work=3_000_000,
              large_work=1_000_000)


def _fields(r):
    return {k: r[k] for k in ("T", "E", "F", "totals", "I")}


def _same(a, b):
    return all(np.array_equal(a[k], b[k]) for k in a)


def test_alone_equals_mix():
    from paper_1403_6126_amd.serve import Server
    wls = _mix()
    with Server(**SERVER) as s:
        hs = [s.submit(wl, keep_I=True) for wl in wls]
        mix = [s.wait(h) for h in hs]
        c = s.counters()
    print("statuses", [(wl.name, r["status"], r["packed"]) for wl, r in zip(wls, mix)],
          c, flush=True)
    assert all(r["status"] == 0 for r in mix)
    assert c["packed_requests"] >= 3 and c["chunk_launches"] >= 5, c
    assert any(r["packed"] for r in mix) and not all(r["packed"] for r in mix)
    for i, wl in enumerate(wls):
        with Server(**SERVER) as s:
            alone = s.wait(s.submit(wl, keep_I=True))
        ok = _same(_fields(alone), _fields(mix[i]))
        print(f"request {i} {wl.name} packed={mix[i]['packed']} same={ok}", flush=True)
        assert ok, i


def test_served_equals_plain_path():
    """Packed and chunked requests give what rt_step gives, bit for bit."""
    import torch

    from paper_1403_6126_amd import rt
    from paper_1403_6126_amd.serve import Server
    from paper_1403_6126_amd.solver import Solver, quadrature_for
    wls = [_mix()[i] for i in (0, 2, 5, 6, 8)]
    with Server(**SERVER) as s:
        hs = [s.submit(wl, keep_I=True) for wl in wls]
        got = [s.wait(h) for h in hs]
    for wl, r in zip(wls, got):
        mu, w = quadrature_for(wl.quad)
        sv = Solver(wl, mu=mu, w=w, I0=torch.zeros((len(w), wl.ncell), dtype=torch.float64,
                                                    device="cuda"))
        rt.rt_equilibrium_intensity(sv.ctx, sv.T, sv.I[0], torch.cuda.current_stream().cuda_stream)
        sv.step(wl.nsteps)
        st = sv.state()
        sv.close()
        ref = dict(T=st["T"], E=st["E"], F=st["F"], totals=st["totals"],
                   I=st["I"].astype(np.float32))
        diffs = {k: float(np.abs(np.asarray(r[k], dtype=np.float64) - ref[k]).max())
                 for k in ref}
        print(wl.name, "packed" if r["packed"] else "chunked", diffs, flush=True)
        assert all(np.array_equal(np.asarray(r[k]), ref[k]) for k in ref), diffs


def test_packed_request_matches_oracle():
    import oracle
    from paper_1403_6126_amd.serve import Server
    wl = _mix()[4]   # 4^3 cells, S4: one workgroup
    with Server(**SERVER) as s:
        r = s.wait(s.submit(wl, keep_I=True))
    assert r["packed"]
    ref = oracle.run(wl, wl.nsteps)
    scale = lambda a: max(np.abs(a).max(), 1e-300)
    errs = dict(E=np.abs(r["E"] - ref.E).max() / scale(ref.E),
                F=np.abs(r["F"] - ref.F).max() / scale(ref.E),
                T=np.abs(r["T"] - ref.T).max() / scale(ref.T))
    print("packed vs oracle", errs, flush=True)
    assert max(errs.values()) <= TOL_MIXED, errs


def test_admission_limits():
    from paper_1403_6126_amd.serve import Server
    wls = _mix()
    # an arena that holds only a few requests at once, and two slots
    kw = dict(SERVER, pool_bytes=600 << 20, max_active=2)
    with Server(**kw) as s:
        hs = [s.submit(wl) for wl in wls]
        res = [s.wait(h) for h in hs]
        c = s.counters()
    assert all(r["status"] == 0 for r in res)
    assert c["peak_active"] <= 2 and c["peak_pool_used"] <= c["pool_bytes"]
    assert c["completed"] == len(wls) and c["pool_used"] == 0
    # admissions follow submission order
    admits = [r["t_admit"] for r in res]
    assert admits == sorted(admits)


def test_submit_validation():
    from paper_1403_6126_amd import rt
    from paper_1403_6126_amd.serve import Server
    wl = _mix()[0]
    with Server(**SERVER) as s:
        wl.courant = 1.5          # beyond the CFL limit
        with pytest.raises(rt.RTError) as ei:
            s.submit(wl)
        assert ei.value.status == rt.RT_ECFL
        wl.courant = 0.5
        wl.nsteps = 0
        with pytest.raises(rt.RTError) as ei:
            s.submit(wl)
        assert ei.value.status == rt.RT_EINVAL
        wl.nsteps = 3
    with Server(**dict(SERVER, pool_bytes=1 << 20)) as s:
        with pytest.raises(rt.RTError) as ei:
            s.submit(_mix()[9])   # footprint beyond the whole arena
        assert ei.value.status == rt.RT_ENOMEM
