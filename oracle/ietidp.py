"""IETI-DP with exact local solves (the D-D variant of Sec. 3.3), FP64.

Written in the notation of Sec. 2-3:

* tearing: every patch keeps its own copy of its coefficients; the
  boundary (Dirichlet) coefficients are dropped (V_0 = H^1_0);
* primal ("strongly enforced") continuity: the values at patch vertices and,
  on request, the averages over patch edges (in 2D the patch sides, the
  choice of the paper's 2D experiments, Sec. 4), or the edge averages alone
  (the paper's 3D choice, Sec. 4; vertex copies are then joined by
  multipliers like every other interface coefficient); C^(k) evaluates them
  on patch k and R_Pi^(k) maps local to global primal unknowns.  A patch
  that touches no Dirichlet boundary has a singular K^(k) (constants); its
  constraints C^(k) remove that kernel, so the saddle-point matrices below
  stay regular (Sec. 3.2, the case of eq. (6) with a semi-definite block);
* the primal basis of W_Pi solves the saddle-point systems of eq. (6) with
  the stiffness K^(k) in place of S^(k) (Pechstein's approach), for every
  local constraint j:  [K C^T; C 0] [phi_j; mu_j] = [0; e_j];
* the coarse matrix S_PiPi = sum_k R^T Phi^T K Phi R is factored densely
  (Cholesky), the direct coarse solve of Sec. 3.3;
* the local Neumann problem in W_Delta, eq. (7), is the same saddle-point
  matrix with right-hand side [g; 0]; so
    K~^{-1} g = sum_k [w_Delta^(k)] + Phi S_PiPi^{-1} Phi^T g,
  the block-diagonal structure S~ = diag(S_DeltaDelta^(k), S_PiPi);
* the jump operator B: one Lagrange multiplier per pair of patches sharing
  a non-primal coefficient (fully redundant), +1 on the lower, -1 on the
  higher patch index; B_D scales each entry by 1 / (number of patches
  holding the coefficient) (multiplicity scaling);
* F = B K~^{-1} B^T, d = B K~^{-1} f (eq. (4)), solved by CG from lambda = 0
  with the scaled Dirichlet preconditioner M^{-1} = B_D S B_D^T, where
  S^(k) = K_GG - K_GI K_II^{-1} K_IG is the Schur complement on the
  interface coefficients of patch k (Sec. 2, last paragraph);
* recovery: u = K~^{-1} (f - B^T lambda).

Everything is plain SciPy: SuperLU factorisations of the saddle-point and
interior matrices, a dense Cholesky factor for S_PiPi.
"""
from __future__ import annotations

import itertools
from typing import List

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .conforming import Layout, assemble_all, layout


def _local_corners(shape) -> List[int]:
    out = []
    dim = len(shape)
    for ends in itertools.product(*[(0, s - 1) for s in shape]):
        idx, stride = 0, 1
        for d in range(dim):
            idx += ends[d] * stride
            stride *= shape[d]
        out.append(idx)
    return out


def _local_edges(shape) -> List[np.ndarray]:
    """Coefficients strictly inside each edge of a patch: the 12 edges of a 3D
    patch, or the 4 sides of a 2D patch (the edges of a 2D decomposition)."""
    if len(shape) == 2:
        out = []
        for free in range(2):
            other = 1 - free
            for e in (0, shape[other] - 1):
                run = np.arange(1, shape[free] - 1)
                idx = run * (1 if free == 0 else shape[0]) + e * (shape[0] if other == 1 else 1)
                out.append(idx.astype(np.int64))
        return out
    assert len(shape) == 3
    out = []
    for free in range(3):
        others = [d for d in range(3) if d != free]
        for ea in (0, shape[others[0]] - 1):
            for eb in (0, shape[others[1]] - 1):
                ijk = [None, None, None]
                ijk[others[0]] = ea
                ijk[others[1]] = eb
                run = np.arange(1, shape[free] - 1)
                idx = np.zeros(len(run), dtype=np.int64)
                strides = [1, shape[0], shape[0] * shape[1]]
                for d in range(3):
                    idx += (run if d == free else ijk[d]) * strides[d]
                out.append(idx)
    return out


class IetiDP:
    """Exact-local IETI-DP for a workload from :mod:`workloads`."""

    def __init__(self, wl, primal: str | None = None, lay: Layout | None = None, systems=None):
        self.wl = wl
        self.lay = lay = layout(wl) if lay is None else lay
        self.systems = systems = assemble_all(wl) if systems is None else systems
        primal = wl.primal if primal is None else primal
        if primal not in ("vertices", "vertices+edges", "edges"):
            raise ValueError(f"unknown primal set {primal!r}")
        N = len(wl.patches)
        self.N = N
        # free (non-boundary) local coefficients of each patch
        self.free = [np.flatnonzero(~lay.boundary[g]) for g in lay.gid]
        self.gfree = [lay.gid[k][self.free[k]] for k in range(N)]
        self.K = [systems[k].K[self.free[k]][:, self.free[k]].tocsc() for k in range(N)]
        self.f = [systems[k].F[self.free[k]] for k in range(N)]
        pos_of = [{int(g): i for i, g in enumerate(self.gfree[k])} for k in range(N)]

        # ---- primal constraints: vertices, then (3D) edge averages
        vertex_g = set()
        for k in range(N):
            for c in _local_corners(lay.shapes[k]):
                g = int(lay.gid[k][c])
                if not lay.boundary[g] and primal != "edges":
                    vertex_g.add(g)
        vertex_g = sorted(vertex_g)
        edges = {}
        if primal in ("vertices+edges", "edges"):
            for k in range(N):
                for loc in _local_edges(lay.shapes[k]):
                    g = lay.gid[k][loc]
                    if lay.boundary[g[0]]:
                        continue
                    edges.setdefault(tuple(sorted(int(v) for v in g)), None)
        edge_keys = sorted(edges, key=lambda t: t[0])
        self.n_pi = len(vertex_g) + len(edge_keys)
        gv_index = {g: i for i, g in enumerate(vertex_g)}
        ge_index = {key: len(vertex_g) + i for i, key in enumerate(edge_keys)}
        self.vertex_g = np.array(vertex_g, dtype=np.int64)
        self.C, self.R = [], []
        for k in range(N):
            rows, Rk = [], []
            nf = len(self.free[k])
            for c in _local_corners(lay.shapes[k]):
                g = int(lay.gid[k][c])
                if g in gv_index:
                    r = np.zeros(nf)
                    r[pos_of[k][g]] = 1.0
                    rows.append(r)
                    Rk.append(gv_index[g])
            if edge_keys:
                for loc in _local_edges(lay.shapes[k]):
                    key = tuple(sorted(int(v) for v in lay.gid[k][loc]))
                    if key in ge_index:
                        r = np.zeros(nf)
                        r[[pos_of[k][int(v)] for v in lay.gid[k][loc]]] = 1.0 / len(loc)
                        rows.append(r)
                        Rk.append(ge_index[key])
            self.C.append(sp.csr_matrix(np.array(rows).reshape(len(rows), nf)))
            self.R.append(np.array(Rk, dtype=np.int64))

        # ---- saddle-point factors (eqs. (6), (7) with K) and the primal basis
        self.saddle, self.Phi = [], []
        S_pp = np.zeros((self.n_pi, self.n_pi))
        for k in range(N):
            nk, ck = self.K[k].shape[0], self.C[k].shape[0]
            A = sp.bmat([[self.K[k], self.C[k].T], [self.C[k], None]], format="csc")
            lu = spla.splu(A)
            self.saddle.append(lu)
            rhs = np.zeros((nk + ck, ck))
            rhs[nk:, :] = np.eye(ck)
            Phi = lu.solve(rhs)[:nk, :] if ck else np.zeros((nk, 0))
            self.Phi.append(Phi)
            Sk = Phi.T @ (self.K[k] @ Phi)
            S_pp[np.ix_(self.R[k], self.R[k])] += Sk
        self.S_pp = S_pp
        self.S_pp_chol = sla.cho_factor(S_pp) if self.n_pi else None

        # ---- Lagrange multipliers (fully redundant) and the jump operators
        copies = {}
        vset = set(vertex_g)
        for k in range(N):
            for i, g in enumerate(self.gfree[k]):
                g = int(g)
                if lay.mult[g] > 1 and g not in vset:
                    copies.setdefault(g, []).append((k, i))
        rows = [[] for _ in range(N)]
        cols = [[] for _ in range(N)]
        vals = [[] for _ in range(N)]
        vald = [[] for _ in range(N)]
        n_lam = 0
        self.lam_dof = []
        for g in sorted(copies):
            cp = sorted(copies[g])
            m = len(cp)
            for a in range(m):
                for b in range(a + 1, m):
                    (ka, ia), (kb, ib) = cp[a], cp[b]
                    rows[ka].append(n_lam); cols[ka].append(ia); vals[ka].append(1.0); vald[ka].append(1.0 / m)
                    rows[kb].append(n_lam); cols[kb].append(ib); vals[kb].append(-1.0); vald[kb].append(-1.0 / m)
                    self.lam_dof.append(g)
                    n_lam += 1
        self.n_lam = n_lam
        self.B = [sp.csr_matrix((vals[k], (rows[k], cols[k])), shape=(n_lam, len(self.free[k]))) for k in range(N)]
        self.BD = [sp.csr_matrix((vald[k], (rows[k], cols[k])), shape=(n_lam, len(self.free[k]))) for k in range(N)]

        # ---- interface / interior split for the scaled Dirichlet preconditioner
        self.G, self.I, self.KII = [], [], []
        self.KGG, self.KGI, self.KIG = [], [], []
        for k in range(N):
            m = lay.mult[self.gfree[k]]
            G = np.flatnonzero(m > 1)
            I = np.flatnonzero(m == 1)
            self.G.append(G)
            self.I.append(I)
            Kk = self.K[k]
            self.KII.append(spla.splu(Kk[I][:, I].tocsc()) if len(I) else None)
            self.KGG.append(Kk[G][:, G])
            self.KGI.append(Kk[G][:, I])
            self.KIG.append(Kk[I][:, G])

    # -------------------------------------------------------------- operators
    def ktilde_inv(self, g: List[np.ndarray]):
        """K~^{-1} g: local constrained solves (eq. (7)) plus the primal part."""
        gpi = np.zeros(self.n_pi)
        for k in range(self.N):
            if len(self.R[k]):
                np.add.at(gpi, self.R[k], self.Phi[k].T @ g[k])
        upi = sla.cho_solve(self.S_pp_chol, gpi) if self.n_pi else gpi
        out = []
        for k in range(self.N):
            nk, ck = self.K[k].shape[0], self.C[k].shape[0]
            w = self.saddle[k].solve(np.concatenate([g[k], np.zeros(ck)]))[:nk]
            if ck:
                w = w + self.Phi[k] @ upi[self.R[k]]
            out.append(w)
        return out, upi

    def apply_F(self, lam: np.ndarray) -> np.ndarray:
        w, _ = self.ktilde_inv([self.B[k].T @ lam for k in range(self.N)])
        return sum(self.B[k] @ w[k] for k in range(self.N))

    def rhs_d(self, with_scale: bool = False):
        """d = B K~^{-1} f; with ``with_scale`` also the largest patch term ||B^(k) w^(k)||,
        against which a cancelling sum is judged to be zero up to rounding."""
        w, _ = self.ktilde_inv(self.f)
        terms = [self.B[k] @ w[k] for k in range(self.N)]
        d = sum(terms)
        if with_scale:
            return d, max(float(np.linalg.norm(t)) for t in terms)
        return d

    def schur_apply(self, k: int, vG: np.ndarray) -> np.ndarray:
        """S^(k) v on the interface coefficients of patch k."""
        out = self.KGG[k] @ vG
        if self.KII[k] is not None:
            out = out - self.KGI[k] @ self.KII[k].solve(self.KIG[k] @ vG)
        return out

    def apply_prec(self, r: np.ndarray) -> np.ndarray:
        z = np.zeros(self.n_lam)
        for k in range(self.N):
            v = self.BD[k].T @ r
            s = np.zeros_like(v)
            s[self.G[k]] = self.schur_apply(k, v[self.G[k]])
            z += self.BD[k] @ s
        return z

    # -------------------------------------------------------------- PCG
    def pcg(self, tol: float = 1e-8, maxit: int = 500):
        """CG on F lambda = d with M^{-1}, zero initial guess, ||r_k|| <= tol ||r_0||."""
        d, scale = self.rhs_d(with_scale=True)
        lam = np.zeros(self.n_lam)
        r = d.copy()
        z = self.apply_prec(r)
        p = z.copy()
        rz = float(r @ z)
        r0 = float(np.linalg.norm(r))
        hist = [r0]
        alphas, betas = [], []
        it = 0
        info_break = False
        if r0 <= 1e-13 * scale:     # d vanishes up to rounding: lambda = 0 solves F lambda = d
            return lam, dict(iterations=0, history=hist, alphas=alphas, betas=betas, breakdown=False)
        while it < maxit:
            q = self.apply_F(p)
            pq = float(p @ q)
            if pq <= 0.0:          # breakdown: d is zero up to rounding (symmetric data)
                info_break = True
                break
            alpha = rz / pq
            lam += alpha * p
            r -= alpha * q
            it += 1
            hist.append(float(np.linalg.norm(r)))
            alphas.append(alpha)
            if hist[-1] <= tol * r0:
                break
            z = self.apply_prec(r)
            rz_new = float(r @ z)
            beta = rz_new / rz
            betas.append(beta)
            rz = rz_new
            p = z + beta * p
        return lam, dict(iterations=it, history=hist, alphas=alphas, betas=betas, breakdown=info_break)

    def solve(self, tol: float = 1e-8, maxit: int = 500):
        """Returns the torn solution (one full coefficient array per patch), lambda and PCG info."""
        lam, info = self.pcg(tol, maxit)
        g = [self.f[k] - self.B[k].T @ lam for k in range(self.N)]
        w, upi = self.ktilde_inv(g)
        parts = []
        for k in range(self.N):
            u = np.zeros(len(self.lay.gid[k]))
            u[self.free[k]] = w[k]
            parts.append(u)
        info["u_pi"] = upi
        return parts, lam, info

    # -------------------------------------------------------------- diagnostics
    def jump_norm(self, parts: List[np.ndarray]) -> float:
        return float(np.linalg.norm(sum(self.B[k] @ parts[k][self.free[k]] for k in range(self.N))))

    @staticmethod
    def lanczos_extremes(info) -> tuple:
        """Extreme eigenvalues of M^{-1}F from the CG coefficients (Lanczos tridiagonal)."""
        a, b = info["alphas"], info["betas"]
        n = len(a)
        if n == 0:
            return (np.nan, np.nan)
        T = np.zeros((n, n))
        for i in range(n):
            T[i, i] = 1.0 / a[i] + (b[i - 1] / a[i - 1] if i > 0 else 0.0)
            if i + 1 < n and i < len(b):
                T[i, i + 1] = T[i + 1, i] = np.sqrt(b[i]) / a[i]
        ev = np.linalg.eigvalsh(T)
        return float(ev[0]), float(ev[-1])
