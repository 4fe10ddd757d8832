"""Pins of the oracle's exact-local IETI-DP against independent facts.

* IETI-DP reproduces the global conforming solution (a reformulation,
  Sec. 2 eqs. (2)-(4)): agreement <= 1e-10 when CG runs to 1e-13;
* continuity of the recovered solution across patches (B u = 0);
* F built column by column equals a brute-force dense F = B K~^{-1} B^T in
  which K~ is the torn stiffness with the primal vertex copies merged
  (no primal basis, no saddle-point solves);
* FETI-DP spectral bound lambda_min(M^{-1} F) >= 1 (dense generalised
  eigenvalues on tiny cases);
* F and M^{-1} symmetric;
* the primal basis satisfies C Phi = I and is K-orthogonal to
  {w : C w = 0} (energy-minimising primal subspace, eq. (6)).
"""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

import workloads as W
from oracle import conforming, ietidp

CASES = [
    W.square_2x2(),
    W.deformed_square((3, 3), [[2, 3, 4], [4, 2, 3]], [[8, 12, 16], [16, 8, 12]], amp_factor=0.8),
    W.unit_cube((3, 3, 2), 2, 4),
    W.unit_cube((2, 3, 2), [[2, 3], [2, 2, 3], [3, 2]], [[4, 6], [4, 4, 6], [6, 4]]),
    W.deformed_square((3, 3), [[2, 3, 4], [4, 2, 3]], [[8, 12, 16], [16, 8, 12]], amp_factor=0.8,
                      primal="vertices+edges", name="deformed3x3_mixed_edges"),
]


@pytest.mark.parametrize("wl", CASES, ids=lambda w: w.name)
def test_matches_global_direct(wl):
    u, lay, systems = conforming.solve_direct(wl)
    ie = ietidp.IetiDP(wl, lay=lay, systems=systems)
    parts, lam, info = ie.solve(tol=1e-13)
    ug = conforming.global_from_torn(lay, parts)
    assert np.linalg.norm(ug - u) <= 1e-10 * np.linalg.norm(u)
    # continuity of the torn solution
    nrm = np.sqrt(sum(float(p @ p) for p in parts))
    assert ie.jump_norm(parts) <= 1e-11 * nrm
    # Ritz values of M^{-1}F from the CG coefficients respect the FETI-DP bound
    if info["iterations"] >= 2:
        lo, hi = ie.lanczos_extremes(info)
        assert lo >= 1 - 1e-8 and hi < 50


@pytest.mark.parametrize("wl", [W.square_2x2(), W.unit_cube((2, 2, 2), 2, 4)], ids=lambda w: w.name)
def test_symmetric_data_gives_zero_dual_rhs(wl):
    """On a mirror-symmetric layout with symmetric f the primal space already
    holds the solution: d vanishes to rounding and lambda = 0."""
    u, lay, systems = conforming.solve_direct(wl)
    ie = ietidp.IetiDP(wl, lay=lay, systems=systems)
    parts, lam, info = ie.solve(tol=1e-10)
    assert info["iterations"] == 0
    assert np.linalg.norm(conforming.global_from_torn(lay, parts) - u) <= 1e-12 * np.linalg.norm(u)


def _dense_F_bruteforce(ie):
    """F = B Q (Q^T K Q)^{-1} Q^T B^T with Q merging the primal vertex copies."""
    N = ie.N
    offs = np.cumsum([0] + [len(f) for f in ie.free])
    ntorn = offs[-1]
    vpos = {int(g): i for i, g in enumerate(ie.vertex_g)}
    # columns: one per non-vertex torn coefficient, then one per primal vertex
    cols = []
    nonvertex = []
    for k in range(N):
        for i, g in enumerate(ie.gfree[k]):
            if int(g) in vpos:
                cols.append(ntorn + vpos[int(g)])
            else:
                cols.append(len(nonvertex))
                nonvertex.append(offs[k] + i)
    nv = len(nonvertex)
    cols = np.array(cols)
    cols[cols >= ntorn] = cols[cols >= ntorn] - ntorn + nv
    Q = sp.csr_matrix((np.ones(ntorn), (np.arange(ntorn), cols)), shape=(ntorn, nv + len(vpos)))
    Kt = sp.block_diag(ie.K, format="csr")
    Bt = sp.hstack(ie.B, format="csr")
    Kw = (Q.T @ Kt @ Q).toarray()
    BQ = (Bt @ Q).toarray()
    return BQ @ np.linalg.solve(Kw, BQ.T)


@pytest.mark.parametrize("wl", [
    W.square_2x2(),
    W.deformed_square((2, 3), [[2, 3], [3, 2, 2]], [[4, 6], [5, 4, 6]], amp_factor=1.0),
    W.unit_cube((2, 2, 2), 2, 3, primal="vertices"),
], ids=lambda w: w.name)
def test_F_equals_bruteforce_and_spectral_bound(wl):
    ie = ietidp.IetiDP(wl)
    n = ie.n_lam
    I = np.eye(n)
    F = np.stack([ie.apply_F(I[:, j]) for j in range(n)], axis=1)
    Fb = _dense_F_bruteforce(ie)
    assert np.abs(F - Fb).max() <= 1e-11 * np.abs(Fb).max()
    assert np.abs(F - F.T).max() <= 1e-12 * np.abs(F).max()
    Minv = np.stack([ie.apply_prec(I[:, j]) for j in range(n)], axis=1)
    assert np.abs(Minv - Minv.T).max() <= 1e-12 * np.abs(Minv).max()
    # restrict to range(B) (fully redundant multipliers make F singular on ker B^T)
    Bt = sp.hstack(ie.B).toarray()
    U, s, _ = np.linalg.svd(Bt, full_matrices=False)
    V = U[:, s > 1e-10 * s[0]]
    ev = sla.eigh(V.T @ F @ V, np.linalg.inv(V.T @ Minv @ V), eigvals_only=True)
    assert ev.min() >= 1 - 1e-10


def test_edge_averages_reduce_condition_number():
    """Vertex + edge-average primal space (the paper's 2D choice) gives a
    smaller spectrum of M^{-1} F than vertices alone, and the same solution."""
    wl = W.deformed_square((4, 4), 2, 8, seed=0)
    u, lay, systems = conforming.solve_direct(wl)
    res = {}
    for prim in ("vertices", "vertices+edges"):
        ie = ietidp.IetiDP(wl, primal=prim, lay=lay, systems=systems)
        parts, lam, info = ie.solve(tol=1e-12)
        assert np.linalg.norm(conforming.global_from_torn(lay, parts) - u) <= 1e-10 * np.linalg.norm(u)
        res[prim] = (ie.n_pi, ie.lanczos_extremes(info))
    assert res["vertices"][0] == 9 and res["vertices+edges"][0] == 9 + 24
    assert res["vertices+edges"][1][0] >= 1 - 1e-8
    assert res["vertices+edges"][1][1] < res["vertices"][1][1]


@pytest.mark.parametrize("wl", [CASES[1], CASES[2], CASES[4]], ids=lambda w: w.name)
def test_primal_basis_energy_minimising(wl):
    ie = ietidp.IetiDP(wl)
    rng = np.random.default_rng(0)
    for k in range(ie.N):
        C = ie.C[k].toarray()
        Phi = ie.Phi[k]
        np.testing.assert_allclose(C @ Phi, np.eye(C.shape[0]), atol=1e-12)
        # random w with C w = 0
        w = rng.standard_normal(C.shape[1])
        w -= C.T @ np.linalg.solve(C @ C.T, C @ w)
        assert np.abs(C @ w).max() < 1e-12
        kw = ie.K[k] @ w
        assert np.abs(Phi.T @ kw).max() <= 1e-10 * np.abs(kw).max() * np.abs(Phi).max() * np.sqrt(len(w))


# the paper's 3D primal choice, edge averages without vertex values (Sec. 4), and its 2D analogue (side
# averages only): the centre patches of a 3x3 square and a 3x3x3 cube touch no Dirichlet boundary, so their
# K is singular and only the constraints fix the constants (eq. (6) with a semi-definite block)
EDGE_ONLY = [
    W.unit_cube((2, 2, 2), 2, 4, primal="edges", name="cube2x2x2_edges"),
    W.unit_cube((3, 3, 2), 2, 4, primal="edges", name="cube3x3x2_edges"),
    W.unit_cube((3, 3, 3), 2, 4, primal="edges", name="cube3x3x3_edges"),
    W.deformed_square((3, 3), [[2, 3, 4], [4, 2, 3]], [[8, 12, 16], [16, 8, 12]], amp_factor=0.8,
                      primal="edges", name="deformed3x3_mixed_sides_only"),
]


@pytest.mark.parametrize("wl", EDGE_ONLY, ids=lambda w: w.name)
def test_edge_only_primal_matches_global_direct(wl):
    u, lay, systems = conforming.solve_direct(wl)
    ie = ietidp.IetiDP(wl, lay=lay, systems=systems)
    assert len(ie.vertex_g) == 0
    floating = [k for k in range(ie.N) if len(ie.free[k]) == len(lay.gid[k])]
    if wl.name.startswith(("cube3x3x3", "deformed3x3")):
        assert len(floating) == 1
        k = floating[0]
        # the floating patch's K has the constants as its kernel; its constraints do not
        one = np.ones(ie.K[k].shape[0])
        assert np.abs(ie.K[k] @ one).max() <= 1e-12 * abs(ie.K[k]).max()
        assert np.allclose(ie.C[k] @ one, 1.0)
    parts, lam, info = ie.solve(tol=1e-13)
    ug = conforming.global_from_torn(lay, parts)
    assert np.linalg.norm(ug - u) <= 1e-10 * np.linalg.norm(u)
    nrm = np.sqrt(sum(float(p @ p) for p in parts))
    assert ie.jump_norm(parts) <= 1e-11 * nrm
    if info["iterations"] >= 2:
        lo, hi = ie.lanczos_extremes(info)
        assert lo >= 1 - 1e-8 and hi < 100


@pytest.mark.parametrize("wl", EDGE_ONLY[2:], ids=lambda w: w.name)
def test_edge_only_primal_basis_and_spectral_bound(wl):
    """C Phi = I and Phi K-orthogonal to {C w = 0} on every patch, floating ones included; the dense
    generalised eigenvalues of (F, M) on range(F) respect the FETI-DP bound >= 1."""
    ie = ietidp.IetiDP(wl)
    rng = np.random.default_rng(1)
    for k in range(ie.N):
        C = ie.C[k].toarray()
        Phi = ie.Phi[k]
        np.testing.assert_allclose(C @ Phi, np.eye(C.shape[0]), atol=1e-12)
        w = rng.standard_normal(C.shape[1])
        w -= C.T @ np.linalg.solve(C @ C.T, C @ w)
        kw = ie.K[k] @ w
        assert np.abs(Phi.T @ kw).max() <= 1e-10 * np.abs(kw).max() * np.abs(Phi).max() * np.sqrt(len(w))
    n = ie.n_lam
    I = np.eye(n)
    F = np.stack([ie.apply_F(I[:, j]) for j in range(n)], axis=1)
    Minv = np.stack([ie.apply_prec(I[:, j]) for j in range(n)], axis=1)
    assert np.abs(F - F.T).max() <= 1e-11 * np.abs(F).max()
    # with edge averages primal the jumps B w of w in W~ have zero edge means, so F vanishes on more than
    # ker B^T: the bound holds on range(F) = B(W~)
    fe, fv = np.linalg.eigh(0.5 * (F + F.T))
    V = fv[:, fe > 1e-10 * fe.max()]
    ev = sla.eigh(V.T @ F @ V, np.linalg.inv(V.T @ Minv @ V), eigvals_only=True)
    assert ev.min() >= 1 - 1e-9
