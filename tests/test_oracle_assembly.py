"""Pins of the oracle's assembly and global direct solve.

* 1D interior rows of mass and stiffness on uniform knots equal the closed
  forms from the cardinal B-spline of degree 2p+1 at the integers
  (mass h B_{2p+1}(k), stiffness -B''_{2p+1}(k) / h), values with Eulerian
  numbers that are fixed by the mathematics, not by the oracle;
* identity-geometry 2D/3D matrices are Kronecker sums of 1D ones;
* K 1 = 0 (pure Neumann) and symmetry, also on curved patches;
* the load vector sums to int f (8 in 2D, 24/pi in 3D for the sine loads);
* polynomial patch test: u = prod x(1-x) lies in the spline space for
  p >= 2, so the Galerkin solution reproduces it to rounding;
* L2 convergence of order p+1 for u = sin sin on the deformed square.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from oracle import assembly, bspline, conforming

CLOSED_FORM = {
    2: (np.array([1, 26, 66, 26, 1]) / 120, np.array([-1 / 6, -1 / 3, 1, -1 / 3, -1 / 6])),
    3: (np.array([1, 120, 1191, 2416, 1191, 120, 1]) / 5040,
        np.array([-1 / 120, -1 / 5, -1 / 8, 2 / 3, -1 / 8, -1 / 5, -1 / 120])),
}


def _identity_patch(dim, n_el, p, lo=0.0, hi=1.0):
    ks = tuple(W.uniform_open_knots(n_el, p) for _ in range(dim))
    axes = [lo + (hi - lo) * bspline.greville(k, p) for k in ks]
    return W.Patch(degree=(p,) * dim, knots=ks, ctrl=assembly.tensor_points(axes))


@pytest.mark.parametrize("p", [2, 3])
@pytest.mark.parametrize("length", [1.0, 0.25])
def test_1d_interior_rows_closed_form(p, length):
    n_el = 12
    patch = _identity_patch(1, n_el, p, 0.0, length)
    s = assembly.assemble_patch(patch)
    h = length / n_el
    mid = (n_el + p) // 2
    Mrow = s.M.toarray()[mid, mid - p:mid + p + 1]
    Krow = s.K.toarray()[mid, mid - p:mid + p + 1]
    np.testing.assert_allclose(Mrow, h * CLOSED_FORM[p][0], rtol=1e-13, atol=1e-16)
    np.testing.assert_allclose(Krow, CLOSED_FORM[p][1] / h, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("dim", [2, 3])
def test_affine_patch_is_kronecker_sum(dim):
    p, n_el = 2, 5
    p1 = assembly.assemble_patch(_identity_patch(1, n_el, p))
    pd = assembly.assemble_patch(_identity_patch(dim, n_el, p))
    K1, M1 = p1.K, p1.M
    terms = []
    for a in range(dim):
        mats = [K1 if d == a else M1 for d in range(dim)]
        terms.append(assembly.kron_dirs(mats))
    Kk = sum(terms)
    assert abs(pd.K - Kk).max() < 1e-13
    assert abs(pd.M - assembly.kron_dirs([M1] * dim)).max() < 1e-15


@pytest.mark.parametrize("wl", [
    W.deformed_square((2, 2), 3, 8, seed=0),
    W.deformed_square((3, 2), [[2, 3, 4], [4, 2]], [[6, 8, 10], [8, 6]], amp_factor=1.0),
    W.unit_cube((2, 1, 1), 2, 3),
])
def test_neumann_kernel_and_symmetry(wl):
    for patch in wl.patches:
        s = assembly.assemble_patch(patch, f=wl.f)
        one = np.ones(s.K.shape[0])
        assert np.abs(s.K @ one).max() < 1e-12 * abs(s.K).max()
        assert abs(s.K - s.K.T).max() < 1e-13 * abs(s.K).max()
        ev = np.linalg.eigvalsh(s.K.toarray())
        assert ev[0] > -1e-12 * ev[-1] and ev[1] > 1e-8 * ev[-1]


@pytest.mark.parametrize("wl,expected", [
    (W.deformed_square((2, 2), 2, 16, seed=0), 8.0),
    (W.deformed_square((3, 3), 3, 8), 8.0),
    (W.unit_cube((2, 2, 2), 2, 6), 24 / np.pi),
])
def test_load_vector_integrates_f(wl, expected):
    """Partition of unity: sum_i f_i = int f (quadrature error only)."""
    total = sum(assembly.assemble_patch(p, f=wl.f).F.sum() for p in wl.patches)
    assert abs(total - expected) < 1e-8 * expected


@pytest.mark.parametrize("wl", [
    W.deformed_square((2, 2), 2, 4, rhs="poly"),
    W.deformed_square((2, 3), [[2, 3], [3, 2, 4]], [[4, 5], [3, 4, 6]], rhs="poly"),
    W.unit_cube((2, 2, 1), 2, 3, rhs="poly"),
])
def test_polynomial_patch_test(wl):
    """u = prod x_i(1 - x_i) is in the spline space: the discrete solution is exact."""
    u, lay, systems = conforming.solve_direct(wl)
    parts = conforming.torn_from_global(lay, u)
    err, nrm = assembly.l2_error(systems, parts, wl.u_exact)
    assert err < 1e-12 * nrm


@pytest.mark.parametrize("p", [2, 3])
def test_l2_convergence_rate(p):
    """h^{p+1} convergence for u = sin(pi x) sin(pi y) on the deformed square."""
    hs, errs = [], []
    for n in (4, 8, 16, 32):
        wl = W.deformed_square((2, 2), p, n, seed=0)
        u, lay, systems = conforming.solve_direct(wl)
        e, nrm = assembly.l2_error(systems, conforming.torn_from_global(lay, u), wl.u_exact)
        hs.append(1.0 / n)
        errs.append(e / nrm)
    slope = np.polyfit(np.log(hs), np.log(errs), 1)[0]
    assert slope >= p + 1 - 0.15, (slope, errs)


def test_global_layout_and_conformity():
    wl = W.deformed_16x16_mixed()
    lay = conforming.layout(wl)
    assert lay.nglobal - lay.boundary.sum() == wl.ndof_global
    assert sum(len(g) for g in lay.gid) == wl.ndof_torn
    # interface coefficients are shared by exactly two patches, vertices by four
    assert set(np.unique(lay.mult)) == {1, 2, 4}


def test_galerkin_coarse_operator_affine():
    """Nested spaces and exact quadrature on affine patches: P^T K_h P = K_2h."""
    for dim, p in [(2, 2), (2, 3), (3, 2)]:
        patch = _identity_patch(dim, 8, p, 0.0, 0.5)
        Kf = assembly.assemble_patch(patch).K
        coarse = [bspline.coarsen_knots(k, p) for k in patch.knots]
        Kc = assembly.assemble_patch(patch, knots=coarse).K
        P = assembly.kron_dirs([sp.csr_matrix(bspline.prolongation(c, f, p)) for c, f in zip(coarse, patch.knots)])
        assert abs(P.T @ Kf @ P - Kc).max() < 1e-12 * abs(Kc).max()
