"""Oracle angle sets (TEST INFRASTRUCTURE ONLY; independent of the GPU
library's own quadrature code).

Section 3 of the paper discretises the sphere into directions n_l with
weights W_l such that J = sum I_l W_l, H = sum n_l I_l W_l,
K = sum n_l n_l I_l W_l, and requires K_ii/J = 1/3 for isotropic I.  The
weights here sum to one (J is the mean intensity).

* 1D slabs: Gauss-Legendre nodes mu on [-1, 1] (ascending), weights halved;
  the direction is (mu, 0, 0).
* 2D/3D: a level-symmetric set of order N (N/2 cosine levels; N(N+2)/8
  directions per octant).  The levels are mu_i^2 = (6 i - 5) / (3 (N - 1)),
  i = 1..N/2, which gives the paper's printed cosines 1/3 and 0.882 for three
  directions per octant and the classical S8 levels for ten.  Directions are
  the permutations (mu_i, mu_j, mu_k) with i + j + k = N/2 + 2; directions
  related by a permutation share one weight, fixed by requiring the exact
  sphere averages of the symmetric even monomials x^2a y^2b z^2c, taken in
  graded order (degree, then single-axis powers first), keeping the first
  independent conditions.

Parity unpinned: the paper cites, but does not print, the tables of its
level-symmetric weights, so these weights are not checked against the
paper's sets; what is pinned is that they reproduce the printed cosines and
the exact sphere averages (sum W = 1, sum W n = 0, sum W n n = 1/3 delta and
the higher even moments the conditions above impose).

Canonical order (shared with the GPU library so tables can be compared
entry by entry): octant o = 0..7 with signs (-1 if o&1, -1 if o&2, -1 if
o&4) on (x, y, z); inside an octant, points by ascending i then j.
"""
from __future__ import annotations

import math

import numpy as np


def gauss_legendre(n: int):
    """Nodes and weights of the n-point Gauss-Legendre rule on [-1, 1] by
    Newton iteration on the Legendre recurrence.  Returns (mu[n,3], w[n])
    with weights normalised to sum 1."""
    if n < 2 or n % 2:
        raise ValueError("Gauss-Legendre order must be even and >= 2")
    x = np.empty(n)
    wt = np.empty(n)
    for i in range(n):
        # initial guess: Chebyshev-like asymptotic root location
        z = math.cos(math.pi * (i + 0.75) / (n + 0.5))
        for _ in range(100):
            p0, p1 = 1.0, z
            for k in range(2, n + 1):
                p0, p1 = p1, ((2 * k - 1) * z * p1 - (k - 1) * p0) / k
            dp = n * (z * p1 - p0) / (z * z - 1.0)
            dz = p1 / dp
            z -= dz
            if abs(dz) < 1e-16:
                break
        p0, p1 = 1.0, z
        for k in range(2, n + 1):
            p0, p1 = p1, ((2 * k - 1) * z * p1 - (k - 1) * p0) / k
        dp = n * (z * p1 - p0) / (z * z - 1.0)
        x[i] = z
        wt[i] = 2.0 / ((1.0 - z * z) * dp * dp)
    order = np.argsort(x)
    x, wt = x[order], wt[order]
    # exact symmetry of the rule
    x = 0.5 * (x - x[::-1])
    wt = 0.5 * (wt + wt[::-1])
    mu = np.zeros((n, 3))
    mu[:, 0] = x
    return mu, wt / 2.0


def _double_factorial_odd(k: int) -> int:
    r = 1
    while k > 1:
        r *= k
        k -= 2
    return r


def _sphere_average(a: int, b: int, c: int) -> float:
    """Average over the unit sphere of x^2a y^2b z^2c."""
    f = _double_factorial_odd
    return f(2 * a - 1) * f(2 * b - 1) * f(2 * c - 1) / f(2 * (a + b + c) + 1)


def level_symmetric(order: int):
    """Level-symmetric set of the given order (even, 2..16).  Returns
    (mu[N,3], w[N]) in the canonical order, weights summing to 1."""
    if order < 2 or order % 2 or order > 16:
        raise ValueError("level-symmetric order must be even in [2, 16]")
    half = order // 2
    lev2 = np.array([(6 * i - 5) / (3.0 * (order - 1)) for i in range(1, half + 1)])
    s = half + 2
    pts = [(i, j, s - i - j) for i in range(1, half + 1) for j in range(1, half + 1)
           if 1 <= s - i - j <= half]
    classes = sorted({tuple(sorted(p)) for p in pts})
    nc = len(classes)
    members = {k: [p for p in pts if tuple(sorted(p)) == k] for k in classes}
    rows, rhs = [], []
    for deg in range(0, 2 * order + 1):
        for a in range(deg, -1, -1):
            for b in range(min(a, deg - a), -1, -1):
                c = deg - a - b
                if c > b:
                    continue
                rows.append([sum(lev2[p[0] - 1] ** a * lev2[p[1] - 1] ** b * lev2[p[2] - 1] ** c
                                 for p in members[k]) for k in classes])
                rhs.append(_sphere_average(a, b, c))
    A = np.array(rows)
    b = np.array(rhs)
    sel = []
    for r in range(len(rows)):
        trial = sel + [r]
        if np.linalg.matrix_rank(A[trial], tol=1e-10) == len(trial):
            sel = trial
        if len(sel) == nc:
            break
    # conditions are per-octant averages: weights of one octant sum to 1
    wcls = np.linalg.solve(A[sel], b[sel])
    if np.any(wcls <= 0):
        raise ValueError(f"order {order}: non-positive weights")
    wmap = dict(zip(classes, wcls))
    mus, ws = [], []
    for o in range(8):
        sg = np.array([-1.0 if o & 1 else 1.0, -1.0 if o & 2 else 1.0, -1.0 if o & 4 else 1.0])
        for p in pts:
            mus.append(sg * np.sqrt([lev2[p[0] - 1], lev2[p[1] - 1], lev2[p[2] - 1]]))
            ws.append(wmap[tuple(sorted(p))] / 8.0)
    mu = np.array(mus)
    w = np.array(ws)
    return mu, w


def angle_set(quad):
    """Angle table for a workload's quadrature spec."""
    kind = quad[0]
    if kind == "gl":
        return gauss_legendre(int(quad[1]))
    if kind == "ls":
        return level_symmetric(int(quad[1]))
    if kind == "table":
        return np.asarray(quad[1], dtype=np.float64), np.asarray(quad[2], dtype=np.float64)
    raise ValueError(f"unknown quadrature {quad!r}")
