"""Pins of the oracle's B-spline layer against facts fixed by the mathematics.

Cox-de Boor bases (Sec. 2): partition of unity, non-negativity, linear
reproduction by Greville coefficients, closed-form cardinal values at knots,
derivatives as limits of difference quotients, nestedness of dyadic
refinement (the canonical embedding used by the multigrid hierarchy), and
Gauss-Legendre exactness.
"""
import numpy as np
import pytest

from oracle import assembly, bspline
from workloads import uniform_open_knots


def _random_open_knots(rng, n_el, p):
    inner = np.sort(rng.uniform(0.05, 0.95, n_el - 1))
    return np.concatenate([np.zeros(p + 1), inner, np.ones(p + 1)])


@pytest.mark.parametrize("p", [1, 2, 3, 4, 7])
@pytest.mark.parametrize("uniform", [True, False])
def test_partition_of_unity_and_positivity(p, uniform):
    rng = np.random.default_rng(p)
    t = uniform_open_knots(9, p) if uniform else _random_open_knots(rng, 9, p)
    x = np.concatenate([rng.uniform(0, 1, 200), [0.0, 1.0]])
    N, dN = bspline.basis(t, p, x, deriv=True)
    assert N.shape == (len(x), len(t) - p - 1)
    np.testing.assert_allclose(N.sum(axis=1), 1.0, atol=1e-14)
    np.testing.assert_allclose(dN.sum(axis=1), 0.0, atol=1e-11)
    assert N.min() >= -1e-15
    # every point sees at most p+1 nonzero functions
    assert (np.count_nonzero(N > 1e-15, axis=1) <= p + 1).all()


@pytest.mark.parametrize("p", [1, 2, 3, 5])
def test_greville_reproduces_linears(p):
    rng = np.random.default_rng(10 + p)
    t = _random_open_knots(rng, 7, p)
    x = rng.uniform(0, 1, 100)
    N = bspline.basis(t, p, x)
    np.testing.assert_allclose(N @ bspline.greville(t, p), x, atol=1e-14)


@pytest.mark.parametrize("p,vals", [
    (1, [1.0]),
    (2, [0.5, 0.5]),
    (3, [1 / 6, 2 / 3, 1 / 6]),
    (4, [1 / 24, 11 / 24, 11 / 24, 1 / 24]),
])
def test_cardinal_values_at_interior_knot(p, vals):
    """Uniform B-splines at an interior knot far from the ends: the values of
    the cardinal B-spline at the integers (Eulerian numbers / p!)."""
    n_el = 12
    t = uniform_open_knots(n_el, p)
    x = np.array([6.0 / n_el])
    N = bspline.basis(t, p, x)[0]
    nz = N[N > 1e-15]
    np.testing.assert_allclose(nz, vals, atol=1e-14)


@pytest.mark.parametrize("p", [2, 3, 4])
def test_derivative_is_difference_quotient_limit(p):
    rng = np.random.default_rng(3)
    t = _random_open_knots(rng, 6, p)
    b = np.unique(t)
    # points well inside knot spans so the central difference does not cross a knot
    x = (b[:-1] + b[1:]) / 2
    h = 1e-6
    _, dN = bspline.basis(t, p, x, deriv=True)
    fd = (bspline.basis(t, p, x + h) - bspline.basis(t, p, x - h)) / (2 * h)
    np.testing.assert_allclose(dN, fd, atol=1e-6 * max(1, np.abs(dN).max()))


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_prolongation_is_exact_refinement(p):
    """A coarse spline and its prolongated coefficients define the same function."""
    rng = np.random.default_rng(20 + p)
    fine = uniform_open_knots(16, p)
    coarse = bspline.coarsen_knots(fine, p)
    np.testing.assert_allclose(coarse, uniform_open_knots(8, p))
    P = bspline.prolongation(coarse, fine, p)
    assert P.shape == (16 + p, 8 + p)
    c = rng.standard_normal(8 + p)
    x = rng.uniform(0, 1, 300)
    np.testing.assert_allclose(bspline.basis(fine, p, x) @ (P @ c), bspline.basis(coarse, p, x) @ c, atol=1e-13)
    # interior columns carry the dyadic subdivision mask binom(p+1, j) / 2^p
    mid = P[:, (8 + p) // 2]
    nz = mid[np.abs(mid) > 1e-14]
    from math import comb
    np.testing.assert_allclose(nz, [comb(p + 1, j) / 2 ** p for j in range(p + 2)], atol=1e-13)


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6])
@pytest.mark.parametrize("graded", [False, True])
def test_prolongation_band_widths(p, graded):
    """Midpoint refinement: a row of the prolongation (one fine coefficient) has at most (p + 1) // 2 + 1
    consecutive nonzero entries, a column (one coarse B-spline) p + 2: the widths the device transfer tables
    hold, also for non-uniform breakpoints."""
    for nel in (6, 8, 12, 16):
        if graded:
            b = np.linspace(0.0, 1.0, nel // 2 + 1) ** 2          # coarse breakpoints, graded
            mids = 0.5 * (b[1:] + b[:-1])
            br = np.sort(np.concatenate([b, mids]))
            fine = np.concatenate([np.zeros(p), br, np.ones(p)])
        else:
            fine = uniform_open_knots(nel, p)
        coarse = bspline.coarsen_knots(fine, p)
        P = bspline.prolongation(coarse, fine, p)
        nz = np.abs(P) > 1e-14
        for row in nz:
            idx = np.nonzero(row)[0]
            assert idx.max() - idx.min() + 1 <= (p + 1) // 2 + 1
            assert len(idx) == idx.max() - idx.min() + 1
        for col in nz.T:
            idx = np.nonzero(col)[0]
            assert idx.max() - idx.min() + 1 <= p + 2


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 8])
def test_gauss_exactness(n):
    x, w = assembly.gauss01(n)
    for k in range(2 * n):
        assert abs(np.dot(w, x ** k) - 1.0 / (k + 1)) < 1e-14
    # degree 2n is not integrated exactly
    assert abs(np.dot(w, x ** (2 * n)) - 1.0 / (2 * n + 1)) > 1e-12
