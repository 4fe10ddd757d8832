"""Tensor-product smoother of the finest multigrid level, 2D (FP64, dense).

TEST INFRASTRUCTURE ONLY, like the rest of this package.

Sec. 4 makes multigrid robust in the spline degree with a smoother on the
finest grid of the subspace-corrected mass smoother kind (Hofreither and
Takacs), modified by a rank-one approximation of the geometry transformation.
The variant defined here, written from that description:

* the metric of the stiffness, G = |det J| J^{-1} J^{-T}, evaluated at the
  (p+1)-point Gauss grid of the patch; only its diagonal g_00, g_11 enters;
* each g_dd (a Q0 x Q1 array, Q_d = Gauss points of direction d) is replaced
  by its best rank-one approximation (leading singular pair):
  g_00 ~ a00 (x) b00, g_11 ~ a11 (x) b11, with the two "mass" factors b00
  and a11 scaled to unit mean over [0, 1] (Gauss weights);
* one-dimensional matrices per direction with those weights:
  A_0 = (a00 N', N'), B_0 = (a11 N, N) on direction 0,
  A_1 = (b11 N', N'), B_1 = (b00 N, N) on direction 1, so that
  K_sep = A_0 (x) B_1 + B_0 (x) A_1 is the stiffness of the separable metric
  (direction 0 fastest, so the Kronecker factors appear as kron(dir1, dir0));
* the smoother operator S = K_sep + c M_sep, M_sep = B_0 (x) B_1,
  c = sigma * mean_d(n_el,d^2) (a mass shift of order h^-2);
* for a local problem whose mode removes some coefficients: sides removed
  from the tensor space direction by direction, removed corners (primal
  vertices) cut afterwards by the mask m:  P r = m S_kept^{-1} m r;
* one smoothing step x <- x + tau P (b - K x), tau = 1 / lambda_max(P K).

The functions below build these objects with plain dense NumPy/SciPy (no
fast diagonalisation): the library's eigenvector factors are checked against
them.  Pins (tests/test_oracle_tensor_smoother.py): K_sep equals the
assembled stiffness on tensor-product geometry maps (where the metric is
diagonal and each diagonal entry separable), the rank-one factors reproduce
an exactly separable array, and the dense solve equals the eigenvector form.
"""
from __future__ import annotations

from typing import List, Sequence, Tuple

import numpy as np
import scipy.linalg as sla

from . import assembly, bspline


def gauss_grid(geo):
    """Gauss points and weights of every direction of the patch's own space."""
    xs, ws = [], []
    for d in range(geo.dim):
        x, w = assembly.element_quadrature(np.asarray(geo.knots[d]), geo.degree[d] + 1)
        xs.append(x)
        ws.append(w)
    return xs, ws


def metric_diagonals(geo) -> Tuple[List[np.ndarray], list, list]:
    """g_dd = |det J| (J^{-1} J^{-T})_dd on the Gauss grid, as Q0 x Q1 arrays (index [q0, q1])."""
    if geo.dim != 2:
        raise ValueError("2D patches only")
    xs, ws = gauss_grid(geo)
    _, J = assembly.geometry_eval(geo, xs)
    det = np.linalg.det(J)
    Ji = np.linalg.inv(J)
    G = np.einsum("qac,qbc->qab", Ji, Ji) * det[:, None, None]
    Q0, Q1 = len(xs[0]), len(xs[1])
    # the grid's flat index runs direction 0 fastest
    g = [G[:, d, d].reshape(Q1, Q0).T.copy() for d in range(2)]
    return g, xs, ws


def rank_one(g: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """Leading singular pair of a positive array, g ~ outer(a, b), both factors positive."""
    u, s, vt = np.linalg.svd(g)
    a = u[:, 0] * s[0]
    b = vt[0].copy()
    if b.sum() < 0:
        a, b = -a, -b
    return a, b


def separable_matrices(geo):
    """(A_0, B_0, A_1, B_1) of the separable metric, with the unit-mean scaling of b00 and a11."""
    g, xs, ws = metric_diagonals(geo)
    a00, b00 = rank_one(g[0])
    a11, b11 = rank_one(g[1])
    m1 = float(ws[1] @ b00)
    b00, a00 = b00 / m1, a00 * m1
    m0 = float(ws[0] @ a11)
    a11, b11 = a11 / m0, b11 * m0
    mats = []
    for d, (ws_d, wm_d) in enumerate(((a00, a11), (b11, b00))):
        N, dN = bspline.basis(np.asarray(geo.knots[d]), geo.degree[d], xs[d], deriv=True)
        N = N.toarray() if hasattr(N, "toarray") else np.asarray(N)
        dN = dN.toarray() if hasattr(dN, "toarray") else np.asarray(dN)
        A = dN.T @ np.diag(ws[d] * ws_d) @ dN
        B = N.T @ np.diag(ws[d] * wm_d) @ N
        mats += [A, B]
    return tuple(mats)


def k_sep(geo) -> np.ndarray:
    """The separable stiffness A_0 (x) B_1 + B_0 (x) A_1 (dense, direction 0 fastest)."""
    A0, B0, A1, B1 = separable_matrices(geo)
    return np.kron(B1, A0) + np.kron(A1, B0)


def shift(geo, sigma: float) -> float:
    nel = [len(np.unique(np.asarray(geo.knots[d]))) - 1 for d in range(2)]
    return sigma * 0.5 * (nel[0] ** 2 + nel[1] ** 2)


def kept_indices(geo, sides: int) -> List[np.ndarray]:
    """Per direction, the coefficients left after removing the masked sides (bit 2d + e: side xi_d = e)."""
    out = []
    for d in range(2):
        M = bspline.n_basis(np.asarray(geo.knots[d]), geo.degree[d])
        keep = np.ones(M, bool)
        if sides >> (2 * d) & 1:
            keep[0] = False
        if sides >> (2 * d + 1) & 1:
            keep[-1] = False
        out.append(np.flatnonzero(keep))
    return out


def smoother_matrix(geo, sides: int, sigma: float) -> Tuple[np.ndarray, np.ndarray]:
    """S = K_sep + c M_sep restricted to the tensor space of kept coefficients; returns (S_kept, flat kept index)."""
    A0, B0, A1, B1 = separable_matrices(geo)
    k0, k1 = kept_indices(geo, sides)
    c = shift(geo, sigma)
    A0, B0 = A0[np.ix_(k0, k0)], B0[np.ix_(k0, k0)]
    A1, B1 = A1[np.ix_(k1, k1)], B1[np.ix_(k1, k1)]
    S = np.kron(B1, A0) + np.kron(A1, B0) + c * np.kron(B1, B0)
    M0 = bspline.n_basis(np.asarray(geo.knots[0]), geo.degree[0])
    flat = (k0[None, :] + M0 * k1[:, None]).ravel()
    return S, flat


def apply(geo, sides: int, mask: np.ndarray, r: np.ndarray, sigma: float) -> np.ndarray:
    """P r = m S_kept^{-1} m r by a dense solve (mask: True where the mode holds a coefficient at zero)."""
    S, flat = smoother_matrix(geo, sides, sigma)
    rr = np.where(mask, 0.0, r)
    y = np.zeros_like(r)
    y[flat] = sla.solve(S, rr[flat], assume_a="pos")
    y[mask] = 0.0
    return y


def apply_eig(geo, sides: int, mask: np.ndarray, r: np.ndarray, sigma: float) -> np.ndarray:
    """The same operator by the eigenvectors of the pairs (A_d, B_d) (fast diagonalisation)."""
    A0, B0, A1, B1 = separable_matrices(geo)
    k0, k1 = kept_indices(geo, sides)
    c = shift(geo, sigma)
    l0, U0 = sla.eigh(A0[np.ix_(k0, k0)], B0[np.ix_(k0, k0)])
    l1, U1 = sla.eigh(A1[np.ix_(k1, k1)], B1[np.ix_(k1, k1)])
    M0 = len(A0)
    M1 = len(A1)
    R = np.where(mask, 0.0, r).reshape(M1, M0)[np.ix_(k1, k0)]
    Z = (U1.T @ R @ U0) / (l1[:, None] + l0[None, :] + c)
    Y = np.zeros((M1, M0))
    Y[np.ix_(k1, k0)] = U1 @ Z @ U0.T
    y = Y.ravel()
    y[mask] = 0.0
    return y


def damping(geo, sides: int, mask: np.ndarray, K: np.ndarray, sigma: float) -> float:
    """lambda_max(P K) on the unmasked coefficients by a dense eigenvalue solve (small patches)."""
    keep = np.flatnonzero(~mask)
    S, flat = smoother_matrix(geo, sides, sigma)
    n = len(mask)
    Sinv = np.zeros((n, n))
    Sinv[np.ix_(flat, flat)] = np.linalg.inv(S)
    PK = Sinv[np.ix_(keep, keep)] @ K[np.ix_(keep, keep)]
    return float(np.max(np.linalg.eigvals(PK).real))
