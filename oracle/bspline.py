"""B-spline bases on open knot vectors (Sec. 2, Cox-de Boor recursion), FP64.

Plain, dense evaluation: every function returns the values of all M basis
functions at every requested point.  Slow and obviously correct.
"""
from __future__ import annotations

import numpy as np


def n_basis(knots: np.ndarray, p: int) -> int:
    return len(knots) - p - 1


def _degree0(knots: np.ndarray, x: np.ndarray) -> np.ndarray:
    """Indicator functions of the knot spans [t_i, t_{i+1}); the right end point
    belongs to the last non-empty span so that the basis is defined on [0, 1]."""
    t = knots
    n0 = len(t) - 1
    N = np.zeros((len(x), n0))
    for i in range(n0):
        if t[i] < t[i + 1]:
            N[:, i] = (x >= t[i]) & (x < t[i + 1])
    last = max(i for i in range(n0) if t[i] < t[i + 1])
    N[x >= t[-1], last] = 1.0
    return N


def basis(knots: np.ndarray, p: int, x, deriv: bool = False):
    """Cox-de Boor: values of N_{i,p}, i = 0..M-1, at points x -> array (len(x), M).

    N_{i,0} = 1 on [t_i, t_{i+1}), and
    N_{i,k}(x) = (x - t_i)/(t_{i+k} - t_i) N_{i,k-1}(x)
               + (t_{i+k+1} - x)/(t_{i+k+1} - t_{i+1}) N_{i+1,k-1}(x),
    with 0/0 read as 0.  With ``deriv`` also returns the first derivatives
    N'_{i,p} = p/(t_{i+p} - t_i) N_{i,p-1} - p/(t_{i+p+1} - t_{i+1}) N_{i+1,p-1}.
    """
    t = np.asarray(knots, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    N = _degree0(t, x)
    prev = N
    for k in range(1, p + 1):
        m = len(t) - 1 - k
        Nk = np.zeros((len(x), m))
        for i in range(m):
            d1 = t[i + k] - t[i]
            d2 = t[i + k + 1] - t[i + 1]
            if d1 > 0:
                Nk[:, i] += (x - t[i]) / d1 * N[:, i]
            if d2 > 0:
                Nk[:, i] += (t[i + k + 1] - x) / d2 * N[:, i + 1]
        prev = N
        N = Nk
    if not deriv:
        return N
    M = n_basis(t, p)
    dN = np.zeros((len(x), M))
    if p > 0:
        for i in range(M):
            d1 = t[i + p] - t[i]
            d2 = t[i + p + 1] - t[i + 1]
            if d1 > 0:
                dN[:, i] += p / d1 * prev[:, i]
            if d2 > 0:
                dN[:, i] -= p / d2 * prev[:, i + 1]
    return N, dN


def greville(knots: np.ndarray, p: int) -> np.ndarray:
    """Greville abscissae xi*_i = (t_{i+1} + ... + t_{i+p}) / p."""
    M = n_basis(knots, p)
    return np.array([np.mean(knots[i + 1:i + p + 1]) for i in range(M)])


def breakpoints(knots: np.ndarray) -> np.ndarray:
    return np.unique(knots)


def coarsen_knots(knots: np.ndarray, p: int) -> np.ndarray:
    """Open knot vector keeping every second breakpoint (the next coarser nested space)."""
    b = breakpoints(knots)
    if (len(b) - 1) % 2:
        raise ValueError("odd number of elements cannot be halved")
    bc = b[::2]
    return np.concatenate([np.full(p + 1, bc[0]), bc[1:-1], np.full(p + 1, bc[-1])])


def prolongation(coarse: np.ndarray, fine: np.ndarray, p: int) -> np.ndarray:
    """Coefficient map of the canonical embedding S_p(coarse) -> S_p(fine).

    The coarse space is a subspace of the fine one, so each coarse basis
    function has exact fine coefficients.  They are found by collocation at
    the fine Greville abscissae, where the fine collocation matrix is
    nonsingular (Schoenberg-Whitney): P = N_f(tau)^{-1} N_c(tau).
    """
    tau = greville(fine, p)
    Af = basis(fine, p, tau)
    Ac = basis(coarse, p, tau)
    P = np.linalg.solve(Af, Ac)
    P[np.abs(P) < 1e-14] = 0.0
    return P


def mixed_mass(tf: np.ndarray, pf: int, tc: np.ndarray, pc: int) -> np.ndarray:
    """Mass matrix between two spline spaces on [0, 1]: M[i, j] = int N_i^{(tf, pf)} N_j^{(tc, pc)} dx, by
    Gauss quadrature with pf + pc + 1 points on every interval between consecutive breakpoints of either
    space (exact for the polynomial products there)."""
    b = np.union1d(breakpoints(tf), breakpoints(tc))
    g, w = np.polynomial.legendre.leggauss(pf + pc + 1)
    g, w = 0.5 * (g + 1.0), 0.5 * w
    xs = np.concatenate([a + (c - a) * g for a, c in zip(b[:-1], b[1:])])
    ws = np.concatenate([(c - a) * w for a, c in zip(b[:-1], b[1:])])
    return basis(tf, pf, xs).T @ (ws[:, None] * basis(tc, pc, xs))


def l2_projection(tf: np.ndarray, pf: int, tc: np.ndarray, pc: int) -> np.ndarray:
    """Coefficient map of the L2 projection from the space (tc, pc) onto the space (tf, pf) on [0, 1]:
    u_f = M_f^{-1} M_fc u_c, M_f the mass matrix of the target space and M_fc the mixed one.  This is the
    transfer between non-nested multigrid levels (degree p on the finest level, degree 1 below, Sec. 4);
    its tensor product over the directions is the parametric projection of a patch."""
    return np.linalg.solve(mixed_mass(tf, pf, tf, pf), mixed_mass(tf, pf, tc, pc))
