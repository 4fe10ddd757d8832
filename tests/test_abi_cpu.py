"""The C-ABI library loads on the CPU and exports every symbol include/ieti.h declares;
host-side planning (no device call) matches the oracle's assembly."""
import ctypes
import os
import re

import numpy as np
import pytest

import workloads as W
from oracle import assembly, bspline
from paper_1705_04531_amd import _abi
from paper_1705_04531_amd.solver import Plan, default_options

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    txt = open(os.path.join(ROOT, "include", "ieti.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(ieti_[a-z_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_abi.LIB_PATH):
        pytest.fail("libieti.so is not built; run __graft_entry__.build()")
    return _abi.lib()


def test_exports_every_declared_symbol(lib):
    raw = ctypes.CDLL(_abi.LIB_PATH)
    syms = _declared_symbols()
    assert len(syms) >= 12
    for s in syms:
        assert hasattr(raw, s), s
        assert s in _abi.SIGNATURES, f"binding lacks {s}"


def test_strerror_and_defaults(lib):
    assert lib.ieti_strerror(_abi.IETI_ENOCONV).decode() == "no convergence"
    o = default_options()
    assert o.tol == 1e-8 and o.inner_tol == 1e-10 and o.prec_vcycles == 2 and o.mg_precision == 64


def _dense_from_stencil(pl, k, level):
    coef = pl.array(_abi.IETI_ARR_STENCIL, k, level)
    offs = pl.array(_abi.IETI_ARR_STENCIL_OFFS, k, level, dtype=np.int32).reshape(-1, 3)
    M = pl.array(_abi.IETI_ARR_SHAPE, k, level, dtype=np.int32)
    n = int(np.prod(M))
    coef = coef.reshape(len(offs), n)
    idx = np.stack(np.meshgrid(*[np.arange(m) for m in M], indexing="ij"), -1).reshape(-1, 3, order="F")
    K = np.zeros((n, n))
    for s, o in enumerate(offs):
        j = idx + o
        ok = np.all((j >= 0) & (j < M), axis=1)
        assert np.all(coef[s, ~ok] == 0)
        ii = np.flatnonzero(ok)
        jj = j[ok, 0] + M[0] * (j[ok, 1] + M[1] * j[ok, 2])
        K[ii, jj] += coef[s, ii]
        if s:
            K[jj, ii] += coef[s, ii]
    return K


@pytest.mark.parametrize("wl", [
    W.square_2x2(),
    W.deformed_square((3, 3), [[2, 3, 4], [4, 2, 3]], [[8, 12, 16], [16, 8, 12]], amp_factor=0.8),
    W.unit_cube((2, 2, 2), 2, 6),
], ids=lambda w: w.name)
def test_plan_matches_oracle_assembly(lib, wl):
    pl = Plan(wl.patches, default_options(primal=3 if wl.dim == 3 else 1))
    sz = pl.sizes()
    assert sz["ndof_torn"] == wl.ndof_torn and sz["ndof_global"] == wl.ndof_global
    for k in range(len(wl.patches)):
        K = _dense_from_stencil(pl, k, 0)
        Ko = assembly.assemble_patch(wl.patches[k]).K.toarray()
        assert np.abs(K - Ko).max() <= 1e-13 * np.abs(Ko).max()
    # coarse levels: rediscretisation of the same geometry on the coarse knots
    nlev = int(pl.array(_abi.IETI_ARR_MASKS, 0, 0, dtype=np.int32)[2])
    for lvl in range(1, nlev):
        p0 = wl.patches[0]
        kn = list(p0.knots)
        for _ in range(lvl):
            kn = [bspline.coarsen_knots(t, p) for t, p in zip(kn, p0.degree)]
        Ko = assembly.assemble_patch(p0, knots=kn).K.toarray()
        K = _dense_from_stencil(pl, 0, lvl)
        assert np.abs(K - Ko).max() <= 1e-13 * np.abs(Ko).max()
        for d in range(wl.dim):
            P = pl.array(_abi.IETI_ARR_PROLONG, 0, (d << 8) | (lvl - 1))
            fine = list(p0.knots)
            for _ in range(lvl - 1):
                fine = [bspline.coarsen_knots(t, p) for t, p in zip(fine, p0.degree)]
            Po = bspline.prolongation(kn[d], fine[d], p0.degree[d])
            assert np.abs(P.reshape(Po.shape) - Po).max() < 1e-13
    xq = pl.quadrature()
    xo = np.concatenate([assembly.quadrature_points(p) for p in wl.patches])
    assert np.abs(xq - xo).max() < 1e-14


def test_plan_errors(lib):
    wl = W.deformed_square((2, 2), 2, 4)
    bad = W.deformed_square((2, 2), 2, 4)
    bad.patches[1] = W.deformed_square((2, 2), 2, 6).patches[1]   # 4 vs 6 elements along a shared side
    with pytest.raises(_abi.IetiError) as e:
        Plan(bad.patches)
    assert e.value.code == _abi.IETI_ENONCONFORMING
    flipped = W.deformed_square((2, 2), 2, 4)
    flipped.patches[0].ctrl = flipped.patches[0].ctrl.copy()
    flipped.patches[0].ctrl[:, 0] *= -1.0        # mirrored patch: det J < 0
    with pytest.raises(_abi.IetiError):
        Plan(flipped.patches)
    with pytest.raises(_abi.IetiError) as e:
        Plan(wl.patches, default_options(mg_precision=16))
    assert e.value.code == _abi.IETI_EINVAL


def _mask_from_bits(shape, sides, corners, mode):
    dim = len(shape)
    idx = np.stack(np.meshgrid(*[np.arange(m) for m in shape], indexing="ij"), -1).reshape(-1, dim, order="F")
    m = np.zeros(len(idx), dtype=bool)
    sb = sides if mode == 0 else (0x3F if dim == 3 else 0xF)
    for d in range(dim):
        m |= (idx[:, d] == 0) & bool(sb >> (2 * d) & 1)
        m |= (idx[:, d] == shape[d] - 1) & bool(sb >> (2 * d + 1) & 1)
    if mode == 0:
        corner = np.all((idx == 0) | (idx == np.array(shape) - 1), axis=1)
        cb = sum(((idx[:, d] == shape[d] - 1).astype(int) << d) for d in range(dim))
        m |= corner & ((corners >> cb) & 1).astype(bool)
    return m


@pytest.mark.parametrize("mode", [0, 1])
def test_band_cholesky_factor(lib, mode):
    """The blocked banded Cholesky data of the exact local solver reproduce the
    masked patch stiffness (oracle assembly): L L^T = K with masked rows and
    columns replaced by the identity."""
    wl = W.deformed_square((2, 2), 3, 6, seed=0)
    pl = Plan(wl.patches, default_options(local_solver=_abi.IETI_LOCAL_EXACT))
    nb = 64
    for k in (0, 3):
        p = wl.patches[k]
        shape = p.shape
        n = int(np.prod(shape))
        b = p.degree[0] + p.degree[1] * shape[0]
        data = pl.array(_abi.IETI_ARR_BAND, k, mode)
        nblk = (n + nb - 1) // nb
        bs = nb * (2 * b + nb)
        assert data.size == nblk * bs
        L = np.zeros((nblk * nb, nblk * nb + b))   # columns shifted by b
        for r in range(nblk):
            blk = data[r * bs:(r + 1) * bs]
            Loff = blk[:nb * b].reshape(nb, b)
            Linv = blk[2 * nb * b:].reshape(nb, nb)
            L[r * nb:(r + 1) * nb, r * nb:r * nb + b] = Loff          # columns r*nb - b .. r*nb - 1
            L[r * nb:(r + 1) * nb, b + r * nb:b + (r + 1) * nb] = np.linalg.inv(Linv)
        Ld = L[:n, b:b + n]
        K = assembly.assemble_patch(p).K.toarray()
        bits = pl.array(_abi.IETI_ARR_MASKS, k, 0, dtype=np.int32)
        m = _mask_from_bits(shape, int(bits[0]), int(bits[1]), mode)
        A = K.copy()
        A[m, :] = 0.0
        A[:, m] = 0.0
        A[m, m] = 1.0
        assert np.abs(Ld @ Ld.T - A).max() <= 1e-12 * np.abs(A).max()


def test_exact_neumann_mg_dirichlet_plan(lib):
    """D-MG plans hold the banded factor of the Neumann problems only and a
    multigrid hierarchy (for the Dirichlet problems); MG plans hold no factor."""
    wl = W.deformed_square((2, 2), 3, 32, seed=0)      # 1225 coefficients per patch: two levels
    pl = Plan(wl.patches, default_options(local_solver=_abi.IETI_LOCAL_EXACT_MG))
    assert pl.sizes()["max_levels"] >= 2
    assert pl.array(_abi.IETI_ARR_BAND, 0, 0).size > 0
    with pytest.raises(_abi.IetiError):          # no Dirichlet factor
        pl.array(_abi.IETI_ARR_BAND, 0, 1)
    pm = Plan(wl.patches, default_options(local_solver=_abi.IETI_LOCAL_MG))
    assert pm.sizes()["max_levels"] == pl.sizes()["max_levels"]
    with pytest.raises(_abi.IetiError):          # no factor at all
        pm.array(_abi.IETI_ARR_BAND, 0, 0)
    with pytest.raises(_abi.IetiError):
        Plan(wl.patches, default_options(local_solver=4))


def test_tensor_smoother_factors_match_oracle(lib):
    """The plan's tensor-smoother data (finest level, modes N and D) against the oracle's separable
    matrices: U_d^T A_d U_d = Lambda_d and U_d^T B_d U_d = I on the coefficients the mode keeps, zero
    rows where it removes them, the mass shift, and tau lambda_max(P K) in [0.99, 1.1] with lambda_max from
    a dense eigenvalue solve of the oracle's smoother (power steps may overshoot it slightly)."""
    from oracle import tensor_smoother as TS
    wl = W.deformed_square((3, 3), [[2, 3, 4], [4, 2, 3]], [[12, 16, 24], [16, 12, 24]], amp_factor=1.0)
    opt = default_options(smoother=_abi.IETI_SMOOTHER_TENSOR, coarse_dofs=0)
    pl = Plan(wl.patches, opt)
    for k in (0, 4, 5):
        geo = wl.patches[k]
        A0, B0, A1, B1 = TS.separable_matrices(geo)
        bits = pl.array(_abi.IETI_ARR_MASKS, k, 0, dtype=np.int32)
        K = assembly.assemble_patch(geo).K.toarray()
        for mode in (0, 1):
            sides = int(bits[0]) if mode == 0 else 0xF
            kept = TS.kept_indices(geo, sides)
            par = pl.array(_abi.IETI_ARR_TENSOR_PARAMS, k, mode)
            assert par[2] == pytest.approx(TS.shift(geo, 0.3), rel=1e-14)
            for d, (A, B) in enumerate(((A0, B0), (A1, B1))):
                Pd = int(par[d])
                U = pl.array(_abi.IETI_ARR_TENSOR_U, k, 256 * mode + d).reshape(Pd, Pd)
                lam = pl.array(_abi.IETI_ARR_TENSOR_LAMBDA, k, 256 * mode + d)
                kk = kept[d]
                nk = len(kk)
                Uk = U[kk][:, :nk]
                Ak, Bk = A[np.ix_(kk, kk)], B[np.ix_(kk, kk)]
                assert np.abs(Uk.T @ Bk @ Uk - np.eye(nk)).max() <= 1e-9
                assert np.abs(Uk.T @ Ak @ Uk - np.diag(lam[:nk])).max() <= 1e-9 * lam[:nk].max()
                rest = np.setdiff1d(np.arange(Pd), kk)
                assert np.all(U[rest] == 0.0) and np.all(U[:, nk:] == 0.0) and np.all(lam[nk:] == 1e300)
            m = _mask_from_bits(geo.shape, int(bits[0]), int(bits[1]), mode)
            lmax = TS.damping(geo, sides, m, K, 0.3)
            assert 0.99 <= par[3] * lmax <= 1.1, (k, mode, par[3] * lmax)


def test_tensor_smoother_options(lib):
    wl = W.deformed_square((2, 2), 2, 8, seed=0)
    with pytest.raises(_abi.IetiError):
        Plan(wl.patches, default_options(smoother=2))
    with pytest.raises(_abi.IetiError):
        Plan(wl.patches, default_options(smoother=_abi.IETI_SMOOTHER_TENSOR, smoother_sigma=0.0))
    pl = Plan(wl.patches, default_options())
    with pytest.raises(_abi.IetiError):         # no tensor data for the Chebyshev smoother
        pl.array(_abi.IETI_ARR_TENSOR_PARAMS, 0, 0)


def test_tensor_smoother_factors_match_oracle_3d(lib):
    """3D plans: the three eigenvector factors per mode against the oracle's separable matrices, the shift
    (sigma times the mean squared element count) and tau."""
    from oracle import tensor_smoother as TS
    wl = W.unit_cube((2, 2, 2), 2, 6)
    pl = Plan(wl.patches, default_options(smoother=_abi.IETI_SMOOTHER_TENSOR, coarse_dofs=0))
    geo = wl.patches[0]
    pairs = TS.separable_pairs(geo)
    bits = pl.array(_abi.IETI_ARR_MASKS, 0, 0, dtype=np.int32)
    K = assembly.assemble_patch(geo).K.toarray()
    for mode in (0, 1):
        sides = int(bits[0]) if mode == 0 else 0x3F
        kept = TS.kept_indices(geo, sides)
        par = pl.array(_abi.IETI_ARR_TENSOR_PARAMS, 0, mode)
        assert par[2] == pytest.approx(TS.shift(geo, 0.3), rel=1e-14) and int(par[4]) == int(par[0])
        for d, (A, B) in enumerate(pairs):
            Pd = int(par[d] if d < 2 else par[4])
            U = pl.array(_abi.IETI_ARR_TENSOR_U, 0, 256 * mode + d).reshape(Pd, Pd)
            lam = pl.array(_abi.IETI_ARR_TENSOR_LAMBDA, 0, 256 * mode + d)
            kk = kept[d]
            nk = len(kk)
            Uk = U[kk][:, :nk]
            assert np.abs(Uk.T @ B[np.ix_(kk, kk)] @ Uk - np.eye(nk)).max() <= 1e-9
            assert np.abs(Uk.T @ A[np.ix_(kk, kk)] @ Uk - np.diag(lam[:nk])).max() <= 1e-9 * lam[:nk].max()
        m = _mask_from_bits(geo.shape, int(bits[0]), int(bits[1]), mode)
        lmax = TS.damping(geo, sides, m, K, 0.3)
        assert 0.99 <= par[3] * lmax <= 1.1, (mode, par[3] * lmax)


@pytest.mark.parametrize("wl", [
    W.unit_cube((3, 3, 3), 2, 8, primal="edges", name="cube3x3x3_edges"),
    W.deformed_square((3, 3), [[2, 3, 4], [4, 2, 3]], [[8, 12, 16], [16, 8, 12]], amp_factor=0.8,
                      primal="edges", name="deformed3x3_sides_only"),
], ids=lambda w: w.name)
def test_edge_only_plan_matches_oracle(lib, wl):
    """The paper's edge-average-only primal set: the plan's primal and multiplier counts equal the oracle's
    (vertex copies joined by fully redundant multipliers); the floating centre patch keeps the exact K on the
    finest level and carries K + 1e-2 M^ (M^ the mass matrix of the parameter domain) on the coarser levels."""
    from oracle import ietidp
    from paper_1705_04531_amd import options_for
    pl = Plan(wl.patches, options_for(wl, coarse_dofs=0))
    sz = pl.sizes()
    ie = ietidp.IetiDP(wl)
    assert sz["n_primal"] == ie.n_pi and sz["n_lambda"] == ie.n_lam
    k = len(wl.patches) // 2                        # the centre patch touches no boundary
    masks = pl.array(_abi.IETI_ARR_MASKS, k, 0, dtype=np.int32)
    assert masks[0] == 0 and masks[1] == 0           # no boundary side, no primal vertex
    p = wl.patches[k]
    Ko = assembly.assemble_patch(p).K.toarray()
    assert np.abs(_dense_from_stencil(pl, k, 0) - Ko).max() <= 1e-13 * np.abs(Ko).max()
    kn = [bspline.coarsen_knots(t, d) for t, d in zip(p.knots, p.degree)]
    Kc = assembly.assemble_patch(p, knots=kn).K.toarray()
    # the parametric mass: the same spline space on the identity map of (0,1)^d
    ident = W.Patch(p.degree, p.knots, np.stack(np.meshgrid(
        *[W.greville(t, d) for t, d in zip(p.knots, p.degree)], indexing="ij"), -1).reshape(-1, wl.dim, order="F"))
    Mc = assembly.assemble_patch(ident, knots=kn).M.toarray()
    K1 = _dense_from_stencil(pl, k, 1)
    assert np.abs(K1 - (Kc + 1e-2 * Mc)).max() <= 1e-12 * np.abs(Kc).max()
    # a boundary patch has no mass shift
    K1b = _dense_from_stencil(pl, 0, 1)
    Kcb = assembly.assemble_patch(wl.patches[0], knots=[bspline.coarsen_knots(t, d) for t, d in
                                                        zip(wl.patches[0].knots, wl.patches[0].degree)]).K.toarray()
    assert np.abs(K1b - Kcb).max() <= 1e-13 * np.abs(Kcb).max()


def test_floating_patch_needs_a_constraint(lib):
    """Without vertices and edge averages a patch with no Dirichlet coefficient has nothing fixing its
    constants: planning refuses it; floating patches with another local solver than MG-MG are refused."""
    from paper_1705_04531_amd import options_for
    wl = W.deformed_square((3, 3), 2, 6, primal="edges")
    with pytest.raises(_abi.IetiError) as e:
        Plan(wl.patches, options_for(wl, primal=0))
    assert e.value.code == _abi.IETI_EINVAL
    with pytest.raises(_abi.IetiError) as e:
        Plan(wl.patches, options_for(wl, local_solver=_abi.IETI_LOCAL_EXACT))
    assert e.value.code == _abi.IETI_ENOTSUP
    Plan(wl.patches, options_for(wl))
