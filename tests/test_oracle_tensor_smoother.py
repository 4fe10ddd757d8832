"""Pins of the oracle's tensor-product smoother (oracle/tensor_smoother.py)
against closed forms and independent routines, not against itself:

* the rank-one factors reproduce an exactly separable array;
* on tensor-product geometry maps x = (phi(xi_0), psi(xi_1)) the metric is
  diagonal with separable entries (g_00 = psi'/phi', g_11 = phi'/psi'), so the
  separable stiffness must equal the stiffness the assembly module builds
  from the full metric; a swapped weight or a transposed Kronecker factor
  fails this for phi != psi;
* the dense solve with S = K_sep + c M_sep equals the eigenvector (fast
  diagonalisation) form, and S is symmetric positive definite.
"""
import numpy as np
import pytest

import workloads as W
from oracle import assembly, bspline
from oracle import tensor_smoother as TS


def _tensor_map_patch(p0, p1, n0, n1, phi, psi):
    k0, k1 = W.uniform_open_knots(n0, p0), W.uniform_open_knots(n1, p1)
    g0, g1 = bspline.greville(k0, p0), bspline.greville(k1, p1)
    X0, X1 = np.meshgrid(phi(g0), psi(g1), indexing="ij")
    ctrl = np.stack([X0.ravel(order="F"), X1.ravel(order="F")], axis=1)
    return W.Patch(degree=(p0, p1), knots=(k0, k1), ctrl=ctrl)


def test_rank_one_of_separable_array():
    rng = np.random.default_rng(3)
    a, b = rng.uniform(0.5, 2.0, 17), rng.uniform(0.5, 2.0, 23)
    g = np.outer(a, b)
    x, y = TS.rank_one(g)
    assert np.abs(np.outer(x, y) - g).max() <= 1e-13 * g.max()
    assert np.all(x > 0) and np.all(y > 0)


@pytest.mark.parametrize("p0,p1,n0,n1", [(2, 2, 6, 6), (3, 2, 8, 5), (2, 4, 5, 7)])
def test_separable_stiffness_equals_assembly_on_tensor_maps(p0, p1, n0, n1):
    phi = lambda t: 0.5 + 1.5 * t + 0.3 * t * t          # noqa: E731
    psi = lambda t: -1.0 + 0.7 * t - 0.2 * np.sin(t)     # noqa: E731  (monotone: psi' >= 0.5)
    geo = _tensor_map_patch(p0, p1, n0, n1, phi, psi)
    K = assembly.assemble_patch(geo).K.toarray()
    Ks = TS.k_sep(geo)
    assert np.abs(Ks - K).max() <= 1e-11 * np.abs(K).max()
    # the identity map as well (affine: constant metric)
    geo_id = _tensor_map_patch(p0, p1, n0, n1, lambda t: t, lambda t: 2.0 * t)
    K = assembly.assemble_patch(geo_id).K.toarray()
    assert np.abs(TS.k_sep(geo_id) - K).max() <= 1e-12 * np.abs(K).max()


def test_separable_stiffness_close_on_deformed_patch():
    """On the deformed square the off-diagonal metric and the non-separable part are small: K_sep is an
    SPD approximation of K within the deformation amplitude."""
    wl = W.deformed_square((2, 2), 3, 8, amp_factor=1.0)
    geo = wl.patches[1]
    K = assembly.assemble_patch(geo).K.toarray()
    Ks = TS.k_sep(geo)
    rel = np.abs(Ks - K).max() / np.abs(K).max()
    assert 1e-4 < rel < 0.3


@pytest.mark.parametrize("sides", [0x0, 0x5, 0xF])
def test_dense_solve_equals_eigenvector_form(sides):
    wl = W.deformed_square((3, 3), [[2, 3, 4], [4, 2, 3]], [[6, 8, 10], [8, 6, 10]], amp_factor=1.0)
    geo = wl.patches[4]
    shape = geo.shape
    n = int(np.prod(shape))
    rng = np.random.default_rng(1)
    r = rng.standard_normal(n)
    idx = np.stack(np.meshgrid(*[np.arange(m) for m in shape], indexing="ij"), -1).reshape(-1, 2, order="F")
    mask = np.all((idx == 0) | (idx == np.array(shape) - 1), axis=1)     # corners cut, as primal vertices
    S, flat = TS.smoother_matrix(geo, sides, 0.3)
    assert np.allclose(S, S.T) and np.linalg.eigvalsh(S).min() > 0
    y1 = TS.apply(geo, sides, mask, r, 0.3)
    y2 = TS.apply_eig(geo, sides, mask, r, 0.3)
    assert np.abs(y1 - y2).max() <= 1e-10 * np.abs(y1).max()
    assert np.all(y1[mask] == 0.0)


def test_rank_one_of_separable_3d_array():
    rng = np.random.default_rng(4)
    x = [rng.uniform(0.5, 2.0, n) for n in (7, 9, 11)]
    g = np.einsum("i,j,k->ijk", *x)
    y = TS.rank_one(g)
    assert np.abs(np.einsum("i,j,k->ijk", *y) - g).max() <= 1e-12 * g.max()


def test_separable_stiffness_equals_assembly_on_3d_tensor_map():
    """x = (phi(xi_0), psi(xi_1), chi(xi_2)): g_00 = psi' chi' / phi' etc. are rank one and the mass factors
    a direction receives from the two other diagonals agree, so K_sep = K."""
    p, n = (2, 3, 2), (4, 3, 5)
    k = [W.uniform_open_knots(n[d], p[d]) for d in range(3)]
    g = [bspline.greville(k[d], p[d]) for d in range(3)]
    phi = lambda t: 0.5 + 1.5 * t + 0.3 * t * t          # noqa: E731
    psi = lambda t: -1.0 + 0.7 * t - 0.2 * np.sin(t)     # noqa: E731
    chi = lambda t: 2.0 + t + 0.25 * t ** 3              # noqa: E731
    X = np.meshgrid(phi(g[0]), psi(g[1]), chi(g[2]), indexing="ij")
    ctrl = np.stack([x.ravel(order="F") for x in X], axis=1)
    geo = W.Patch(degree=p, knots=tuple(k), ctrl=ctrl)
    K = assembly.assemble_patch(geo).K.toarray()
    assert np.abs(TS.k_sep(geo) - K).max() <= 1e-11 * np.abs(K).max()
