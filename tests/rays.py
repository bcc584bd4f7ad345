"""Steady-state intensity along straight rays, for pins of the beam
problems: with the temperature held fixed, no scattering and no flow, the
steady transfer equation along direction n is dI/ds = sigma_a (B - I), whose
solution back to the boundary is, for fields constant over each short
segment of length ds,

    I = I_in e^{-tau_total} + sum_k B_k (1 - e^{-sigma_k ds}) e^{-tau_k},

tau_k the optical depth between the point and segment k (Section 2: the
emission of the gas is B = T^4/(4 pi) in code units).  This is a direct
quadrature of the formal solution, independent of the discrete scheme."""
import numpy as np

import workloads as W

FOUR_PI = 4.0 * np.pi


def ray_intensity(x, y, n, sigma, B, entry, box, ds=2e-4):
    """Steady intensity at points (x, y) (arrays) in direction n = (nx, ny).

    sigma(x, y), B(x, y): absorption coefficient and emission of the gas;
    entry(face, x, y) -> incoming intensity where the backward ray leaves
    the box (face 'left', 'right', 'bottom' or 'top'); box = ((x0, x1),
    (y0, y1))."""
    x = np.asarray(x, dtype=np.float64).copy()
    y = np.asarray(y, dtype=np.float64).copy()
    (x0, x1), (y0, y1) = box
    tau = np.zeros_like(x)
    acc = np.zeros_like(x)
    alive = np.ones(x.shape, dtype=bool)
    face = np.empty(x.shape, dtype=object)
    ex, ey = x.copy(), y.copy()
    while alive.any():
        xm = x - 0.5 * ds * n[0]
        ym = y - 0.5 * ds * n[1]
        xn = x - ds * n[0]
        yn = y - ds * n[1]
        out = (xn < x0) | (xn > x1) | (yn < y0) | (yn > y1)
        # the last segment is cut at the face
        frac = np.ones_like(x)
        for val, coord, comp in ((x0, x, 0), (x1, x, 0), (y0, y, 1), (y1, y, 1)):
            if n[comp] != 0.0:
                t = (coord - val) / (ds * n[comp])
                hit = (t >= 0.0) & (t < frac)
                frac = np.where(hit, t, frac)
        step = np.where(out, frac * ds, ds)
        s = sigma(xm, ym)
        a = np.where(alive, s * step, 0.0)
        acc += np.where(alive, B(xm, ym) * (-np.expm1(-a)) * np.exp(-tau), 0.0)
        tau += a
        newly = alive & out
        if newly.any():
            fx = x[newly] - step[newly] * n[0]
            fy = y[newly] - step[newly] * n[1]
            ex[newly], ey[newly] = fx, fy
            eps = 1e-12
            f = np.where(fx <= x0 + eps, "left", np.where(fx >= x1 - eps, "right",
                         np.where(fy <= y0 + eps, "bottom", "top")))
            face[newly] = f
        alive &= ~out
        x, y = xn, yn
    inc = np.array([entry(f, a, b) for f, a, b in zip(face.ravel(), ex.ravel(), ey.ravel())])
    return acc + inc.reshape(acc.shape) * np.exp(-tau)


# ---------------------------------------- the shadow problem (Section 5.8)
def _centres(wl):
    xs = -0.5 + (np.arange(wl.n[0]) + 0.5) * wl.dx[0]
    ys = -0.3 + (np.arange(wl.n[1]) + 0.5) * wl.dx[1]
    X, Y = np.meshgrid(xs, ys)
    return X.ravel(), Y.ravel()


def _rmin(X, Y, n):
    """Smallest ellipse radius r = x^2/a^2 + y^2/b^2 on the ray back from each
    point in direction -n, inside the box."""
    s = np.linspace(0.0, 1.2, 600)[:, None]
    px, py = X[None] - s * n[0], Y[None] - s * n[1]
    inside = (px >= -0.5) & (px <= 0.5) & (py >= -0.3) & (py <= 0.3)
    return np.where(inside, (px / 0.1) ** 2 + (py / 0.06) ** 2, np.inf).min(axis=0)


def classify(wl):
    """(lit, umbra) masks: lit cells have both beam rays well clear of the
    cloud (r > 3, where rho - rho0 < 1e-8) and lie three cells inside the
    box; umbra cells, right of the cloud, have both beam rays through its
    core (r < 0.8, where sigma_a > 1e4)."""
    mu = np.asarray(wl.quad[1])
    X, Y = _centres(wl)
    up, down = wl.meta["beams"]
    ru, rd = _rmin(X, Y, mu[up, :2]), _rmin(X, Y, mu[down, :2])
    inner = (np.abs(X) < 0.5 - 3 * wl.dx[0]) & (np.abs(Y) < 0.3 - 3 * wl.dx[1])
    return (ru > 3.0) & (rd > 3.0) & inner, (ru < 0.8) & (rd < 0.8) & (X > 0.1)


def ray_energy(wl, cells, ds=2e-3):
    """E_r = 4 pi sum_m w_m I_m of the ray solution at the given cells."""
    mu, w = np.asarray(wl.quad[1]), np.asarray(wl.quad[2])
    g = wl.ghost(mu)
    X, Y = _centres(wl)
    sig = lambda x, y: W.shadow_density(x, y) ** 5.5          # T^-3.5 rho^2, T = 1/rho
    B = lambda x, y: W.shadow_density(x, y) ** -4 / FOUR_PI    # T^4 / (4 pi)
    tables = {"left": g[(0, 0)], "bottom": g[(1, 0)], "top": g[(1, 1)]}
    E = np.zeros(len(cells))
    for m in range(len(w)):
        def entry(face, a, b, m=m):  # the copy face sees the background
            return tables[face][m] if face in tables else wl.meta["background"]
        E += FOUR_PI * w[m] * ray_intensity(X[cells], Y[cells], mu[m, :2], sig, B, entry,
                                            wl.meta["box"], ds=ds)
    return E


# ------------------------------------ the crossing beams (Section 5.4)
def beam_stats(wl, I):
    """Per-row statistics of the crossing beams from the intensities
    I (nang, ncell): the x-flux-weighted row flux 4 pi sum_m w_m mu_y I_m dx,
    the flux injected through the bottom face, and for each beam direction
    its centroid along x (circular mean over the periodic axis) and its
    variance about it, row by row."""
    mu, w = np.asarray(wl.quad[1]), np.asarray(wl.quad[2])
    nx, ny = wl.n[0], wl.n[1]
    I = np.asarray(I).reshape(len(w), ny, nx)
    xs = (np.arange(nx) + 0.5) * wl.dx[0]
    ys = (np.arange(ny) + 0.5) * wl.dx[1]
    row = FOUR_PI * np.einsum("m,m,mji->j", w, mu[:, 1], I) * wl.dx[0]
    injected = FOUR_PI * wl.meta["beam"] * wl.dx[0] * sum(
        w[m] * mu[m, 1] * wl.meta["window_cells"][k] for k, m in enumerate(wl.meta["beams"]))
    ang = 2.0 * np.pi * xs
    beams = []
    for k, m in enumerate(wl.meta["beams"]):
        cx = np.arctan2((I[m] * np.sin(ang)).sum(1), (I[m] * np.cos(ang)).sum(1)) / (2 * np.pi)
        cx %= 1.0
        d = (xs[None, :] - cx[:, None] + 0.5) % 1.0 - 0.5
        var = (I[m] * d ** 2).sum(1) / I[m].sum(1)
        # straight line from the window centre at 45 degrees, wrapped
        expect = (wl.meta["centres"][k] + np.sign(mu[m, 0]) * ys) % 1.0
        off = (cx - expect + 0.5) % 1.0 - 0.5
        beams.append(dict(centroid_error=off, var=var))
    return dict(ys=ys, row_flux=row, injected=injected, beams=beams)
