"""Pins of the oracle's final-residual measure and of its Lanczos spectrum estimate.

* ``conforming.global_residual`` (the FP64 assembled residual ||F - K u|| / ||F||
  of the conforming system (Sec. 1 eq. (1), Sec. 2), used for the recovered u):
  - the polynomial patch test: u = x(1-x)y(1-y) lies in the spline space of
    affine patches of degree >= 2, and Gauss quadrature integrates every term
    exactly, so u is the Galerkin solution.  Its B-spline coefficients come from
    the blossom (polar form) of x - x^2 at the knots, with no linear solve;
    the residual of that u is at rounding level;
  - u = 0 gives exactly 1;
  - one interior coefficient perturbed by eps gives eps ||K e_i|| / ||F||, with
    the column K e_i in closed form: the Kronecker sum K1 (x) M1 + M1 (x) K1 of
    the cardinal degree-2 rows (h/120 [1, 26, 66, 26, 1], [-1/6, -1/3, 1, -1/3,
    -1/6] / h), in which h cancels;
  - opposite perturbations of the two copies of an interface coefficient cancel
    in the average of the copies.
* ``IetiDP.lanczos_extremes``: the Ritz values of M^{-1} F from the CG
  coefficients lie inside the spectrum of the dense generalised eigenproblem
  on range(B), and the largest one equals the largest eigenvalue.
"""
import itertools

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

import workloads as W
from oracle import conforming, ietidp


def _blossom_coeffs(t_phys: np.ndarray, p: int) -> np.ndarray:
    """B-spline coefficients of g(x) = x - x^2: the blossom of g at (t_{i+1}, ..., t_{i+p})."""
    m = len(t_phys) - p - 1
    out = np.empty(m)
    for i in range(m):
        a = t_phys[i + 1:i + p + 1]
        lin = a.mean()
        quad = sum(a[j] * a[l] for j, l in itertools.combinations(range(p), 2)) / (p * (p - 1) / 2)
        out[i] = lin - quad
    return out


def _patch_test_parts(wl):
    parts = []
    for pt in wl.patches:
        coef = []
        for d in range(2):
            x = pt.ctrl[:, d]
            x0, x1 = x.min(), x.max()
            coef.append(_blossom_coeffs(x0 + (x1 - x0) * pt.knots[d], pt.degree[d]))
        parts.append(np.outer(coef[1], coef[0]).ravel())
    return parts


def _affine_patch_test(p=2, n=8):
    return W.deformed_square((2, 2), p, n, rhs="poly", name=f"poly2x2_p{p}_n{n}")


def test_residual_of_exact_spline_solution_is_rounding():
    for p in (2, 3):
        wl = _affine_patch_test(p)
        parts = _patch_test_parts(wl)
        r = conforming.global_residual(wl, parts)
        assert r <= 1e-13, (p, r)


def test_residual_of_zero_is_one():
    wl = _affine_patch_test()
    parts = [np.zeros(p.ndof) for p in wl.patches]
    assert abs(conforming.global_residual(wl, parts) - 1.0) <= 1e-15


def test_residual_of_single_perturbation_closed_form():
    wl = _affine_patch_test(2, 8)
    K, F, lay, _ = conforming.global_system(wl)
    normF = np.linalg.norm(F[~lay.boundary])
    k1 = np.array([-1 / 6, -1 / 3, 1.0, -1 / 3, -1 / 6])
    m1 = np.array([1.0, 26.0, 66.0, 26.0, 1.0]) / 120.0
    col = np.outer(k1, m1) + np.outer(m1, k1)       # 5x5 stencil of an interior column, h cancels
    expected_col_norm = np.linalg.norm(col)
    parts = _patch_test_parts(wl)
    # patch 0 interior coefficient (4, 5): its 5x5 neighbourhood lies inside the patch, away from the boundary
    M0 = wl.patches[0].shape[0]
    eps = 1e-3
    parts[0][5 * M0 + 4] += eps
    r = conforming.global_residual(wl, parts)
    assert abs(r - eps * expected_col_norm / normF) <= 1e-9 * r


def test_residual_averages_interface_copies():
    wl = _affine_patch_test(2, 8)
    parts = _patch_test_parts(wl)
    lay = conforming.layout(wl)
    # a coefficient shared by patches 0 and 1 (their common side), not on the boundary
    shared = np.intersect1d(lay.gid[0], lay.gid[1])
    g = int([s for s in shared if not lay.boundary[s]][0])
    i0 = int(np.flatnonzero(lay.gid[0] == g)[0])
    i1 = int(np.flatnonzero(lay.gid[1] == g)[0])
    parts[0][i0] += 0.25
    parts[1][i1] -= 0.25
    assert conforming.global_residual(wl, parts) <= 1e-13
    parts[1][i1] += 0.25            # now the mean moves by 0.125: the residual must see it
    assert conforming.global_residual(wl, parts) > 1e-4


def test_lanczos_extremes_against_dense_spectrum():
    rng = np.random.default_rng(3)
    wl = W.deformed_square((2, 3), [[2, 3], [3, 2, 2]], [[4, 6], [5, 4, 6]], amp_factor=1.0)
    wl.f, wl.u_exact = W.sine_series_rhs(rng.standard_normal((3, 3)))
    ie = ietidp.IetiDP(wl)
    n = ie.n_lam
    eye = np.eye(n)
    F = np.stack([ie.apply_F(eye[:, j]) for j in range(n)], axis=1)
    Minv = np.stack([ie.apply_prec(eye[:, j]) for j in range(n)], axis=1)
    Bt = sp.hstack(ie.B).toarray()
    U, s, _ = np.linalg.svd(Bt, full_matrices=False)
    V = U[:, s > 1e-10 * s[0]]
    ev = sla.eigh(V.T @ F @ V, np.linalg.inv(V.T @ Minv @ V), eigvals_only=True)
    lam, info = ie.pcg(tol=1e-15, maxit=200)
    assert info["iterations"] >= 5
    lo, hi = ie.lanczos_extremes(info)
    assert ev[0] - 1e-10 <= lo <= ev[-1] + 1e-10
    assert abs(hi - ev[-1]) <= 1e-8 * ev[-1]
    assert lo <= ev[0] + 1e-2 * (ev[-1] - ev[0])
