"""Pins of the oracle's angle sets (paper Section 3)."""
import numpy as np
import pytest

from oracle.quadrature import gauss_legendre, level_symmetric
from golden_values import golden

ORDERS = [2, 4, 6, 8, 10, 12, 14, 16]
COUNTS = {2: 8, 4: 24, 6: 48, 8: 80, 10: 120, 12: 168, 14: 224, 16: 288}


def _sets():
    out = [("gl", n) + gauss_legendre(n) for n in (2, 4, 16, 32, 288)]
    out += [("ls", o) + level_symmetric(o) for o in ORDERS]
    return out


@pytest.mark.parametrize("kind,n,mu,w", _sets())
def test_quadrature_identities(kind, n, mu, w):
    # sum w = 1, sum w n = 0, sum w n n = delta/3 (Section 3: K_ii/J = 1/3
    # for isotropic I with any number of angles)
    assert abs(w.sum() - 1.0) <= 1e-15
    assert np.abs(w @ mu).max() <= 1e-15
    K = np.einsum("m,mi,mj->ij", w, mu, mu)
    if kind == "ls":
        assert np.abs(K - np.eye(3) / 3).max() <= 1e-15
        assert np.abs(np.linalg.norm(mu, axis=1) - 1).max() <= 1e-15
    else:
        assert abs(K[0, 0] - 1 / 3) <= 1e-15
    assert (w > 0).all()


@pytest.mark.parametrize("n", [2, 4, 8, 16, 64])
def test_gauss_legendre_matches_numpy(n):
    mu, w = gauss_legendre(n)
    x, wt = np.polynomial.legendre.leggauss(n)
    assert np.abs(mu[:, 0] - x).max() <= 2e-15
    assert np.abs(w - wt / 2).max() <= 2e-15
    assert np.all(mu[:, 1:] == 0)


def test_level_symmetric_counts():
    for o in ORDERS:
        mu, w = level_symmetric(o)
        assert len(w) == COUNTS[o]


def test_s4_matches_paper_printed_cosines():
    # Section 5.2 (Fig. beamingmap caption): with three angles per octant the
    # two distinct polar cosines are 0.333 and 0.882.
    mu, w = level_symmetric(4)
    vals = np.unique(np.round(np.abs(mu), 12))
    assert np.allclose(vals, [1 / 3, np.sqrt(7) / 3], atol=1e-12)
    printed = golden("sec5_2_moving_medium.json")["mu_z_of_the_two_ray_families"]
    assert np.allclose(vals, printed, atol=5e-4)                   # three printed digits
    assert np.allclose(w, 1 / 24)


def test_s8_is_classical_level_set():
    # ten directions per octant: levels mu^2 = 1/21, 7/21, 13/21, 19/21 and
    # the even single-axis moments up to mu^8 integrated exactly
    mu, w = level_symmetric(8)
    lev = np.unique(np.round(mu[:, 0] ** 2, 12))
    assert np.allclose(lev, np.array([1, 7, 13, 19]) / 21)
    for k in range(0, 5):
        exact = 1.0 / (2 * k + 1)
        assert abs(w @ mu[:, 0] ** (2 * k) - exact) < 1e-14


def test_canonical_order_octants():
    mu, w = level_symmetric(8)
    per = len(w) // 8
    for o in range(8):
        blk = mu[o * per:(o + 1) * per]
        sg = [-1 if o & 1 else 1, -1 if o & 2 else 1, -1 if o & 4 else 1]
        assert np.all(np.sign(blk) == sg)


def _dfact(k):
    """(k)!! for odd k >= -1 ((-1)!! = 1)."""
    out = 1
    while k > 1:
        out *= k
        k -= 2
    return out


@pytest.mark.parametrize("order", [4, 6, 8, 10, 12, 14, 16])
def test_level_symmetric_even_moments_exact(order):
    # Section 3 asks the angle set to reproduce the angular moments of an
    # isotropic field.  The sphere average of x^2a y^2b z^2c is
    # (2a-1)!!(2b-1)!!(2c-1)!!/(2a+2b+2c+1)!!; a level-symmetric set of order
    # N integrates every such monomial of degree up to N-2 exactly, so a
    # wrong class weight at any order fails one of these.
    mu, w = level_symmetric(order)
    assert (w > 0).all()
    worst = 0.0
    for deg in range(0, order - 1, 2):
        for a in range(0, deg // 2 + 1):
            for b in range(0, deg // 2 - a + 1):
                c = deg // 2 - a - b
                got = w @ (mu[:, 0] ** (2 * a) * mu[:, 1] ** (2 * b) * mu[:, 2] ** (2 * c))
                exact = (_dfact(2 * a - 1) * _dfact(2 * b - 1) * _dfact(2 * c - 1)
                         / _dfact(2 * (a + b + c) + 1))
                worst = max(worst, abs(got - exact))
    assert worst <= 1e-14, worst
    # the odd moments vanish by the octant symmetry
    assert abs(w @ (mu[:, 0] ** 3 * mu[:, 1])) <= 1e-15
