"""Galerkin assembly of one B-spline patch (Sec. 1 eq. (1), Sec. 2), FP64.

Stiffness  K_ij = int_Omega grad N_i . grad N_j dx
           = sum_q w_q |det J| (J^{-T} grad^ N_i) . (J^{-T} grad^ N_j),
load       f_i  = int_Omega f N_i dx = sum_q w_q |det J| f(G(xi_q)) N^_i(xi_q),
mass       M_ij = int_Omega N_i N_j dx,
with N_i = N^_i o G^{-1} (pull-back) and (p+1) Gauss-Legendre points per
element and direction (the paper does not state its rule; this is the
reading used everywhere in this project).

The discretisation space and the geometry are passed separately so that the
same geometry can be discretised on coarser nested knot vectors.
Dof numbering: direction 0 fastest, i = i0 + M0 (i1 + M1 i2).
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List, Sequence

import numpy as np
import scipy.sparse as sp

from . import bspline


def gauss01(n: int):
    """n-point Gauss-Legendre rule on [0, 1]."""
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def element_quadrature(knots: np.ndarray, npts: int):
    """Gauss points and weights of every non-empty knot span, span-major order."""
    b = bspline.breakpoints(knots)
    g, gw = gauss01(npts)
    xs, ws = [], []
    for a, c in zip(b[:-1], b[1:]):
        xs.append(a + (c - a) * g)
        ws.append((c - a) * gw)
    return np.concatenate(xs), np.concatenate(ws)


def kron_dirs(mats: Sequence):
    """Tensor product over directions, direction 0 fastest in rows and columns."""
    out = sp.csr_matrix(mats[0])
    for m in mats[1:]:
        out = sp.kron(sp.csr_matrix(m), out, format="csr")
    return out


def kron_vec(vecs: Sequence[np.ndarray]) -> np.ndarray:
    out = np.asarray(vecs[0])
    for v in vecs[1:]:
        out = np.kron(v, out)
    return out


def tensor_points(xs: Sequence[np.ndarray]) -> np.ndarray:
    """All points of a tensor grid, direction 0 fastest, shape (n, dim)."""
    mesh = np.meshgrid(*xs, indexing="ij")
    return np.stack([m.ravel(order="F") for m in mesh], axis=1)


def geometry_eval(geo, xs: Sequence[np.ndarray]):
    """G and its Jacobian J[q, c, a] = d x_c / d xi_a on the tensor grid ``xs``."""
    dim = geo.dim
    B, D = [], []
    for d in range(dim):
        b, db = bspline.basis(geo.knots[d], geo.degree[d], xs[d], deriv=True)
        B.append(b)
        D.append(db)
    Bfull = kron_dirs(B)
    x = Bfull @ geo.ctrl
    J = np.zeros((x.shape[0], dim, dim))
    for a in range(dim):
        Ga = kron_dirs([D[d] if d == a else B[d] for d in range(dim)])
        J[:, :, a] = Ga @ geo.ctrl
    return x, J


@dataclass
class PatchSystem:
    K: sp.csr_matrix          # stiffness (no boundary condition applied)
    F: np.ndarray | None      # load vector
    M: sp.csr_matrix          # physical mass matrix
    shape: tuple              # basis functions per direction
    x_qp: np.ndarray          # physical quadrature points (n_qp, dim)
    wdet: np.ndarray          # w_q |det J_q|
    Bq: sp.csr_matrix         # basis values at the quadrature points (n_qp, ndof)


def assemble_patch(geo, knots: Sequence[np.ndarray] | None = None, degree: Sequence[int] | None = None,
                   f=None) -> PatchSystem:
    """Stiffness, mass and load of the space S(knots, degree) on the geometry ``geo``."""
    dim = geo.dim
    knots = list(geo.knots) if knots is None else list(knots)
    degree = list(geo.degree) if degree is None else list(degree)
    xs, ws = [], []
    for d in range(dim):
        x, w = element_quadrature(knots[d], degree[d] + 1)
        xs.append(x)
        ws.append(w)
    xq, J = geometry_eval(geo, xs)
    det = np.linalg.det(J)
    if np.any(det <= 0):
        raise ValueError("geometry map is not orientation preserving at a quadrature point")
    Jinv = np.linalg.inv(J)                       # Jinv[q, a, c] = d xi_a / d x_c
    wdet = kron_vec(ws) * det
    Gm = np.einsum("qac,qbc->qab", Jinv, Jinv) * wdet[:, None, None]
    Bv, Dv = [], []
    for d in range(dim):
        b, db = bspline.basis(knots[d], degree[d], xs[d], deriv=True)
        Bv.append(b)
        Dv.append(db)
    Bq = kron_dirs(Bv)
    grads = [kron_dirs([Dv[d] if d == a else Bv[d] for d in range(dim)]) for a in range(dim)]
    K = None
    for a in range(dim):
        for b in range(dim):
            term = grads[a].T @ sp.diags(Gm[:, a, b]) @ grads[b]
            K = term if K is None else K + term
    K = sp.csr_matrix(K)
    M = sp.csr_matrix(Bq.T @ sp.diags(wdet) @ Bq)
    F = None if f is None else Bq.T @ (wdet * f(xq))
    shape = tuple(bspline.n_basis(knots[d], degree[d]) for d in range(dim))
    return PatchSystem(K=K, F=F, M=M, shape=shape, x_qp=xq, wdet=wdet, Bq=sp.csr_matrix(Bq))


def quadrature_points(geo) -> np.ndarray:
    """Physical quadrature points of the patch's own space, direction 0 fastest,
    element-major within each direction (the order f must be given in)."""
    xs = [element_quadrature(geo.knots[d], geo.degree[d] + 1)[0] for d in range(geo.dim)]
    x, _ = geometry_eval(geo, xs)
    return x


def l2_error(sys_list: List[PatchSystem], u_list: List[np.ndarray], u_exact) -> tuple:
    """(||u_h - u||_L2, ||u||_L2) by the patches' own quadrature."""
    err2 = 0.0
    nrm2 = 0.0
    for s, u in zip(sys_list, u_list):
        uh = s.Bq @ u
        ue = u_exact(s.x_qp)
        err2 += float(np.sum(s.wdet * (uh - ue) ** 2))
        nrm2 += float(np.sum(s.wdet * ue ** 2))
    return np.sqrt(err2), np.sqrt(nrm2)
