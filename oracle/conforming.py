"""The global conforming Galerkin system and its sparse direct solution, FP64.

IETI-DP in every variant (Sec. 2 eqs. (2)-(4), Sec. 3) is a reformulation of
the conforming problem: find u_h in V_h cap H^1_0 with a(u_h, v) = <F, v>
for all v (Sec. 1 eq. (1)).  Its solution is therefore the reference every
IETI-DP result is compared with.

The workloads place patches on a regular grid of the unit square/cube with
matching spline spaces along shared sides, so the global numbering is the
tensor product of per-direction numberings in which neighbouring patches
share their first/last layer of coefficients (C^0 coupling across sides).
Dirichlet dofs are the first and last global layer in every direction.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .assembly import PatchSystem, assemble_patch


@dataclass
class Layout:
    dim: int
    grid: tuple
    pos: List[tuple]            # grid position of each patch
    shapes: List[tuple]         # basis functions per direction of each patch
    gshape: tuple               # global coefficient grid
    gid: List[np.ndarray]       # local -> global flat index, per patch
    boundary: np.ndarray        # bool over global dofs: on the boundary (u = 0)
    mult: np.ndarray            # number of patches holding each global dof

    @property
    def nglobal(self) -> int:
        return int(np.prod(self.gshape))


def _unravel(k: int, grid) -> tuple:
    out = []
    for g in grid:
        out.append(k % g)
        k //= g
    return tuple(out)


def layout(wl) -> Layout:
    dim, grid = wl.dim, tuple(wl.grid)
    pos = [_unravel(k, grid) for k in range(len(wl.patches))]
    shapes = [p.shape for p in wl.patches]
    per_dir = []
    for d in range(dim):
        m = {}
        for ps, sh in zip(pos, shapes):
            if m.setdefault(ps[d], sh[d]) != sh[d]:
                raise ValueError("non-conforming patch grid")
        per_dir.append([m[c] for c in range(grid[d])])
    offs = []
    gshape = []
    for d in range(dim):
        o = [0]
        for c in range(grid[d] - 1):
            o.append(o[-1] + per_dir[d][c] - 1)
        offs.append(o)
        gshape.append(o[-1] + per_dir[d][-1])
    gid = []
    for ps, sh in zip(pos, shapes):
        axes = [offs[d][ps[d]] + np.arange(sh[d]) for d in range(dim)]
        mesh = np.meshgrid(*axes, indexing="ij")
        flat = np.zeros(mesh[0].size, dtype=np.int64)
        stride = 1
        for d in range(dim):
            flat += mesh[d].ravel(order="F") * stride
            stride *= gshape[d]
        gid.append(flat)
    n = int(np.prod(gshape))
    coords = np.stack(np.meshgrid(*[np.arange(s) for s in gshape], indexing="ij"), axis=-1)
    coords = coords.reshape(-1, dim, order="F")
    boundary = np.zeros(n, dtype=bool)
    for d in range(dim):
        boundary |= (coords[:, d] == 0) | (coords[:, d] == gshape[d] - 1)
    mult = np.zeros(n, dtype=np.int64)
    for g in gid:
        mult[g] += 1
    # the geometry must be watertight: shared coefficients carry the same control point
    ref = np.full((n, dim), np.nan)
    for p, g in zip(wl.patches, gid):
        seen = ~np.isnan(ref[g, 0])
        if np.any(seen) and not np.allclose(ref[g[seen]], p.ctrl[seen], atol=1e-12, rtol=0):
            raise ValueError("patches do not meet along a shared side")
        ref[g] = p.ctrl
    return Layout(dim, grid, pos, shapes, tuple(gshape), gid, boundary, mult)


def assemble_all(wl) -> List[PatchSystem]:
    return [assemble_patch(p, f=wl.f) for p in wl.patches]


def global_system(wl, lay: Layout | None = None, systems: List[PatchSystem] | None = None):
    """Sum of the patch matrices and loads in the global numbering (no boundary condition)."""
    lay = layout(wl) if lay is None else lay
    systems = assemble_all(wl) if systems is None else systems
    n = lay.nglobal
    rows, cols, vals = [], [], []
    F = np.zeros(n)
    for s, g in zip(systems, lay.gid):
        c = s.K.tocoo()
        rows.append(g[c.row])
        cols.append(g[c.col])
        vals.append(c.data)
        np.add.at(F, g, s.F)
    K = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))
    return K, F, lay, systems


def solve_direct(wl, lay: Layout | None = None, systems=None):
    """Conforming solution with u = 0 on the boundary, by sparse LU (SuperLU).

    Returns the global coefficient vector (boundary entries zero), the layout
    and the patch systems.
    """
    K, F, lay, systems = global_system(wl, lay, systems)
    free = np.flatnonzero(~lay.boundary)
    Kf = K[free][:, free].tocsc()
    u = np.zeros(lay.nglobal)
    u[free] = spla.splu(Kf).solve(F[free])
    return u, lay, systems


def torn_from_global(lay: Layout, u: np.ndarray) -> List[np.ndarray]:
    return [u[g].copy() for g in lay.gid]


def global_from_torn(lay: Layout, parts: List[np.ndarray]) -> np.ndarray:
    """Mean of the patch copies of every global coefficient."""
    acc = np.zeros(lay.nglobal)
    for g, v in zip(lay.gid, parts):
        np.add.at(acc, g, v)
    return acc / np.maximum(lay.mult, 1)


def global_residual(wl, u_parts: List[np.ndarray], lay: Layout | None = None, systems=None) -> float:
    """||F - K u||_2 / ||F||_2 on the free global dofs, for a torn u (copies averaged)."""
    K, F, lay, systems = global_system(wl, lay, systems)
    u = global_from_torn(lay, u_parts)
    free = ~lay.boundary
    r = (F - K @ u)[free]
    return float(np.linalg.norm(r) / np.linalg.norm(F[free]))
