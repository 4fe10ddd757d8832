"""Tensor-product smoother of the finest multigrid level (FP64, dense).

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
* one smoothing step x <- x + tau P (b - K x), tau = 1 / lambda_max(P K);
* in 3D the same with three diagonals, each fitted by a rank-one three-way
  product; a direction's mass weight is the geometric mean of the two unit-mean
  factors the other diagonals give it (one mass matrix per direction, as the
  Kronecker sum K_sep = A_0 (x) B_1 (x) B_2 + B_0 (x) A_1 (x) B_2 + B_0 (x) B_1 (x) A_2
  requires), c = sigma * mean_d n_el,d^2.

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
    """g_dd = |det J| (J^{-1} J^{-T})_dd on the Gauss grid, as arrays indexed [q0, q1(, q2)]."""
    xs, ws = gauss_grid(geo)
    _, J = assembly.geometry_eval(geo, xs)
    det = np.linalg.det(J)
    Ji = np.linalg.inv(J)
    G = np.einsum("qac,qbc->qab", Ji, Ji) * det[:, None, None]
    Q = tuple(len(x) for x in xs)
    # the grid's flat index runs direction 0 fastest
    g = [G[:, d, d].reshape(Q, order="F").copy() for d in range(geo.dim)]
    return g, xs, ws


def rank_one(g: np.ndarray):
    """Best rank-one approximation of a positive array, all factors positive.

    2D: the leading singular pair, returned as (a, b) with g ~ outer(a, b).  3D: alternating least-squares
    updates of one factor with the other two fixed (the higher-order power method), returned as a list of
    three factors with g ~ x0 (x) x1 (x) x2."""
    if g.ndim == 2:
        u, s, vt = np.linalg.svd(g)
        a = u[:, 0] * s[0]
        b = vt[0].copy()
        if b.sum() < 0:
            a, b = -a, -b
        return a, b
    x = [np.ones(n) for n in g.shape]
    for _ in range(500):
        old = [v.copy() for v in x]
        x[0] = np.einsum("ijk,j,k->i", g, x[1], x[2]) / ((x[1] @ x[1]) * (x[2] @ x[2]))
        x[1] = np.einsum("ijk,i,k->j", g, x[0], x[2]) / ((x[0] @ x[0]) * (x[2] @ x[2]))
        x[2] = np.einsum("ijk,i,j->k", g, x[0], x[1]) / ((x[0] @ x[0]) * (x[1] @ x[1]))
        if max(np.abs(v - o).max() / np.abs(v).max() for v, o in zip(x, old)) <= 1e-15:
            break
    return x


def separable_pairs(geo) -> List[Tuple[np.ndarray, np.ndarray]]:
    """[(A_d, B_d)] per direction: A_d weighted by the stiffness factor of g_dd, B_d by the (geometric mean
    of the) unit-mean mass factors the other diagonals contribute to direction d."""
    g, xs, ws = metric_diagonals(geo)
    dim = geo.dim
    f = []
    for d in range(dim):
        x = list(rank_one(g[d]))
        for e in range(dim):
            if e != d:
                m = float(ws[e] @ x[e])
                x[e] = x[e] / m
                x[d] = x[d] * m
        f.append(x)
    pairs = []
    for e in range(dim):
        wm = np.prod([f[d][e] for d in range(dim) if d != e], axis=0) ** (1.0 / (dim - 1))
        N, dN = bspline.basis(np.asarray(geo.knots[e]), geo.degree[e], xs[e], deriv=True)
        N = N.toarray() if hasattr(N, "toarray") else np.asarray(N)
        dN = dN.toarray() if hasattr(dN, "toarray") else np.asarray(dN)
        pairs.append((dN.T @ np.diag(ws[e] * f[e][e]) @ dN, N.T @ np.diag(ws[e] * wm) @ N))
    return pairs


def separable_matrices(geo):
    """2D: (A_0, B_0, A_1, B_1)."""
    (A0, B0), (A1, B1) = separable_pairs(geo)
    return A0, B0, A1, B1


def _kron_dirs(mats):
    """Kronecker product with direction 0 fastest."""
    out = mats[0]
    for m in mats[1:]:
        out = np.kron(m, out)
    return out


def k_sep(geo) -> np.ndarray:
    """The separable stiffness sum_d B (x) .. A_d .. (x) B (dense, direction 0 fastest)."""
    pairs = separable_pairs(geo)
    dim = geo.dim
    return sum(_kron_dirs([pairs[e][0] if e == d else pairs[e][1] for e in range(dim)]) for d in range(dim))


def shift(geo, sigma: float) -> float:
    nel = [len(np.unique(np.asarray(geo.knots[d]))) - 1 for d in range(geo.dim)]
    return sigma * float(np.mean(np.square(nel)))


def kept_indices(geo, sides: int) -> List[np.ndarray]:
    """Per direction, the coefficients left after removing the masked sides (bit 2d + e: side xi_d = e)."""
    out = []
    for d in range(geo.dim):
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
    pairs = separable_pairs(geo)
    dim = geo.dim
    kk = kept_indices(geo, sides)
    c = shift(geo, sigma)
    A = [pairs[d][0][np.ix_(kk[d], kk[d])] for d in range(dim)]
    B = [pairs[d][1][np.ix_(kk[d], kk[d])] for d in range(dim)]
    S = sum(_kron_dirs([A[e] if e == d else B[e] for e in range(dim)]) for d in range(dim)) + c * _kron_dirs(B)
    M = [bspline.n_basis(np.asarray(geo.knots[d]), geo.degree[d]) for d in range(dim)]
    grids = np.meshgrid(*kk, indexing="ij")
    flat = grids[0].copy()
    stride = 1
    for d in range(1, dim):
        stride *= M[d - 1]
        flat = flat + stride * grids[d]
    return S, flat.ravel(order="F")


def apply(geo, sides: int, mask: np.ndarray, r: np.ndarray, sigma: float) -> np.ndarray:
    """P r = m S_kept^{-1} m r by a dense solve (mask: True where the mode holds a coefficient at zero)."""
    S, flat = smoother_matrix(geo, sides, sigma)
    rr = np.where(mask, 0.0, r)
    y = np.zeros_like(r)
    y[flat] = sla.solve(S, rr[flat], assume_a="pos")
    y[mask] = 0.0
    return y


def apply_eig(geo, sides: int, mask: np.ndarray, r: np.ndarray, sigma: float) -> np.ndarray:
    """The same operator by the eigenvectors of the pairs (A_d, B_d) (fast diagonalisation), 2D."""
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
