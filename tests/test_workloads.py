"""The serving stream's requests are well-posed for the method: the oracle
advances a sample of them (small grids, a few steps) with every temperature
Newton solve converging to a positive root."""
import numpy as np

import workloads as W


def test_config4_requests_are_well_posed(orc):
    reqs = W.config4_requests(120)
    done = 0
    for r in reqs:
        if np.prod(r["shape"]) > 400:
            continue
        wl = W.request_workload(dict(r, nsteps=min(r["nsteps"], 6)), precision="fp64")
        st = orc.run(wl, wl.nsteps)
        # (intensities may dip below zero next to large contrasts: the centred
        # part of the interface flux, weighted 1 - alpha, is not positive)
        assert np.all(st.T > 0) and st.newton_max <= 8, r
        done += 1
    assert done >= 10


def test_config4_request_shapes():
    reqs = W.config4_requests(400)
    cells = np.array([np.prod(r["shape"]) for r in reqs])
    assert cells.min() >= 8 and cells.max() <= 2 * 128 ** 3
    for r in reqs:
        wl = W.request_workload(dict(r, shape=(4,) * r["ndim"]), precision="mixed")
        assert wl.dx[0] == W.configs.REQUEST_DX
        assert abs(wl.courant * np.sqrt(r["ndim"]) - 0.5) < 1e-15
        nang = r["quad"][1] if r["quad"][0] == "gl" else r["quad"][1] * (r["quad"][1] + 2)
        assert 16 <= nang <= 288
