"""Seeded synthetic multipatch Poisson workloads.

Every input of the IETI-DP solver and of the CPU oracle comes from here:
patch knot vectors, geometry control points, the right-hand side ``f`` (a
function of the physical coordinates) and the exact solution that goes with
it.  Both sides consume the same objects.

This module holds none of the solver's arithmetic.  Geometry control points
are placed at the images of the Greville abscissae (means of ``p``
consecutive knots) under an explicit smooth map; that is a definition of the
spline geometry, not an interpolation, so no B-spline evaluation happens
here.  Because open knot vectors put the first and last Greville abscissa on
the parameter boundary, the control points of a patch side depend only on
points of that side, so neighbouring patches with matching knots along a
shared side meet without gaps.

Model problem: -Lap u = f in Omega, u = 0 on the boundary (weak form, Sec. 1,
eq. (1)).  Multipatch B-spline geometry and discretisation: Sec. 2.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, List, Sequence, Tuple

import numpy as np

__all__ = [
    "Patch", "Workload", "Request", "uniform_open_knots", "greville",
    "grid_patches", "sinsin_rhs", "sine_series_rhs", "polynomial_rhs",
    "square_2x2", "deformed_8x8", "deformed_16x16_mixed", "cube_4x4x4",
    "deformed_square", "unit_cube", "serving_stream", "sub_block", "CONFIGS",
]


@dataclass
class Patch:
    """One tensor-product B-spline patch.

    ``knots[i]`` is the open knot vector of direction ``i`` on [0, 1] and
    ``ctrl`` holds ``prod_i M_i`` control points (``M_i = len(knots[i]) -
    degree[i] - 1``), one row per basis function, direction 0 fastest.
    """
    degree: Tuple[int, ...]
    knots: Tuple[np.ndarray, ...]
    ctrl: np.ndarray

    @property
    def dim(self) -> int:
        return len(self.degree)

    @property
    def shape(self) -> Tuple[int, ...]:
        return tuple(len(t) - p - 1 for t, p in zip(self.knots, self.degree))

    @property
    def n_el(self) -> Tuple[int, ...]:
        return tuple(len(np.unique(t)) - 1 for t in self.knots)

    @property
    def ndof(self) -> int:
        return int(np.prod(self.shape))


@dataclass
class Workload:
    """A complete solver input: patches, right-hand side and solver choices."""
    name: str
    dim: int
    grid: Tuple[int, ...]            # patches per direction; patch k = i0 + P0*i1 (+ P0*P1*i2)
    patches: List[Patch]
    f: Callable[[np.ndarray], np.ndarray]        # f(x), x of shape (n, dim)
    u_exact: Callable[[np.ndarray], np.ndarray]
    local_solver: str = "mg"         # "exact" (banded Cholesky) or "mg" (inexact, multigrid)
    mg_precision: int = 64           # 64 or 32 (multigrid arithmetic)
    primal: str = "vertices"         # "vertices" or "vertices+edges" (edge averages; in 2D the patch sides)
    tol: float = 1e-8                # outer PCG: ||r_k||_2 <= tol ||r_0||_2
    inner_tol: float = 1e-10         # local Neumann solves inside F
    seed: int | None = None
    description: str = ""
    extra: dict = field(default_factory=dict)

    @property
    def ndof_torn(self) -> int:
        return sum(p.ndof for p in self.patches)

    @property
    def ndof_global(self) -> int:
        """Conforming dofs with the boundary (Dirichlet) dofs removed."""
        tot = 1
        for d in range(self.dim):
            per = self.extra["dofs_per_dir"][d]   # list of M for each patch index along d
            tot *= sum(per) - (len(per) - 1) - 2
        return tot


@dataclass
class Request:
    """One request of the serving stream: arrival offset (units of 1/rate) and its workload."""
    index: int
    arrival_unit: float
    workload: Workload


def uniform_open_knots(n_el: int, p: int) -> np.ndarray:
    """Open (p+1-fold end knots) uniform knot vector on [0, 1] with n_el elements."""
    inner = np.arange(1, n_el, dtype=np.float64) / n_el
    return np.concatenate([np.zeros(p + 1), inner, np.ones(p + 1)])


def greville(knots: np.ndarray, p: int) -> np.ndarray:
    """Greville abscissae: mean of the p knots strictly inside each basis function's support."""
    m = len(knots) - p - 1
    if p == 0:
        return 0.5 * (knots[:m] + knots[1:m + 1])
    return np.array([knots[i + 1:i + p + 1].mean() for i in range(m)])


# ----------------------------------------------------------------- geometry maps

def _deform_square(amp: float) -> Callable[[np.ndarray], np.ndarray]:
    """x -> x + amp sin(2 pi x0) sin(2 pi x1) (1, 1); identity on the boundary of [0,1]^2."""
    def phi(x: np.ndarray) -> np.ndarray:
        s = amp * np.sin(2 * np.pi * x[:, 0]) * np.sin(2 * np.pi * x[:, 1])
        return x + s[:, None]
    return phi


def _identity(x: np.ndarray) -> np.ndarray:
    return x.copy()


def grid_patches(grid: Sequence[int], n_el: Sequence[Sequence[int]], deg: Sequence[Sequence[int]],
                 phi: Callable[[np.ndarray], np.ndarray]) -> List[Patch]:
    """Patches on a regular grid of the unit square/cube, mapped by ``phi``.

    ``n_el[d][c]`` and ``deg[d][c]`` give elements and degree of direction
    ``d`` for all patches with grid index ``c`` along ``d``, so every shared
    side carries the same spline space from both sides.
    """
    dim = len(grid)
    patches = []
    for flat in range(int(np.prod(grid))):
        idx = []
        r = flat
        for d in range(dim):
            idx.append(r % grid[d])
            r //= grid[d]
        ps = tuple(int(deg[d][idx[d]]) for d in range(dim))
        ks = tuple(uniform_open_knots(int(n_el[d][idx[d]]), ps[d]) for d in range(dim))
        gs = [greville(ks[d], ps[d]) for d in range(dim)]
        # reference point of every control point: affine patch map of its Greville point
        axes = [(idx[d] + gs[d]) / grid[d] for d in range(dim)]
        mesh = np.meshgrid(*axes, indexing="ij")
        # direction 0 fastest: flatten in Fortran order
        ref = np.stack([m.ravel(order="F") for m in mesh], axis=1)
        patches.append(Patch(degree=ps, knots=ks, ctrl=np.ascontiguousarray(phi(ref))))
    return patches


def _dofs_per_dir(grid, n_el, deg):
    return [[int(n_el[d][c]) + int(deg[d][c]) for c in range(grid[d])] for d in range(len(grid))]


# ----------------------------------------------------------------- right-hand sides

def sinsin_rhs(dim: int):
    """f = dim pi^2 prod sin(pi x_i), exact solution u = prod sin(pi x_i) on the unit square/cube."""
    def u(x):
        return np.prod(np.sin(np.pi * x), axis=1)

    def f(x):
        return dim * np.pi ** 2 * np.prod(np.sin(np.pi * x), axis=1)
    return f, u


def sine_series_rhs(coef: np.ndarray):
    """f = sum_{a,b} c_ab sin(a pi x) sin(b pi y); u = sum c_ab sin sin / (pi^2 (a^2 + b^2))."""
    coef = np.asarray(coef, dtype=np.float64)
    na, nb = coef.shape

    def f(x):
        out = np.zeros(x.shape[0])
        for a in range(1, na + 1):
            sa = np.sin(a * np.pi * x[:, 0])
            for b in range(1, nb + 1):
                out += coef[a - 1, b - 1] * sa * np.sin(b * np.pi * x[:, 1])
        return out

    def u(x):
        out = np.zeros(x.shape[0])
        for a in range(1, na + 1):
            sa = np.sin(a * np.pi * x[:, 0])
            for b in range(1, nb + 1):
                out += coef[a - 1, b - 1] * sa * np.sin(b * np.pi * x[:, 1]) / (np.pi ** 2 * (a * a + b * b))
        return out
    return f, u


def polynomial_rhs(dim: int):
    """u = prod x_i (1 - x_i), f = -Lap u = 2 sum_i prod_{j != i} x_j (1 - x_j)."""
    def u(x):
        return np.prod(x * (1 - x), axis=1)

    def f(x):
        q = x * (1 - x)
        out = np.zeros(x.shape[0])
        for i in range(dim):
            out += 2 * np.prod(np.delete(q, i, axis=1), axis=1)
        return out
    return f, u


# ----------------------------------------------------------------- workloads

def deformed_square(grid=(2, 2), p=2, n_el=16, amp_factor: float | None = None, seed: int | None = None,
                    rhs: str = "sinsin", **kw) -> Workload:
    """2D patches on the unit square, optionally deformed by x + 0.05 xi sin sin (1,1).

    With ``amp_factor=None`` and ``seed=None`` the map is the identity.  With a
    seed, ``xi ~ U(0.5, 1)`` is the first draw of ``default_rng(seed)``.
    ``p`` and ``n_el`` may be ints or per-direction, per-grid-index lists.
    """
    rng = None
    xi = 0.0
    if seed is not None:
        rng = np.random.default_rng(seed)
        xi = float(rng.uniform(0.5, 1.0))
    if amp_factor is not None:
        xi = float(amp_factor)
    phi = _deform_square(0.05 * xi) if xi != 0.0 else _identity
    grid = tuple(grid)
    nel = [[n_el] * grid[d] if np.isscalar(n_el) else list(n_el[d]) for d in range(2)]
    deg = [[p] * grid[d] if np.isscalar(p) else list(p[d]) for d in range(2)]
    if rhs == "sinsin":
        f, u = sinsin_rhs(2)
    elif rhs == "poly":
        f, u = polynomial_rhs(2)
    else:
        raise ValueError(rhs)
    patches = grid_patches(grid, nel, deg, phi)
    wl = Workload(name=kw.pop("name", f"square{grid[0]}x{grid[1]}"), dim=2, grid=grid, patches=patches,
                  f=f, u_exact=u, seed=seed, extra={"xi": xi, "dofs_per_dir": _dofs_per_dir(grid, nel, deg)},
                  **kw)
    return wl


def unit_cube(grid=(2, 2, 2), p=2, n_el=6, rhs: str = "sinsin", **kw) -> Workload:
    """3D patches on the unit cube with identity geometry maps."""
    grid = tuple(grid)
    nel = [[n_el] * grid[d] if np.isscalar(n_el) else list(n_el[d]) for d in range(3)]
    deg = [[p] * grid[d] if np.isscalar(p) else list(p[d]) for d in range(3)]
    if rhs == "sinsin":
        f, u = sinsin_rhs(3)
    elif rhs == "poly":
        f, u = polynomial_rhs(3)
    else:
        raise ValueError(rhs)
    patches = grid_patches(grid, nel, deg, _identity)
    kw.setdefault("primal", "vertices+edges")
    return Workload(name=kw.pop("name", f"cube{grid[0]}x{grid[1]}x{grid[2]}"), dim=3, grid=grid,
                    patches=patches, f=f, u_exact=u, extra={"dofs_per_dir": _dofs_per_dir(grid, nel, deg)},
                    **kw)


def square_2x2() -> Workload:
    """Unit square, 2x2 identity patches, p=2, 16x16 elements each, exact local solves."""
    return deformed_square((2, 2), 2, 16, name="square2x2_p2_n16", local_solver="exact", mg_precision=64,
                           description="2D Poisson, 2x2 affine patches, p=2, 16^2 elements, exact local solves")


def deformed_8x8(seed: int = 0) -> Workload:
    """Deformed square, 8x8 patches, p=3, 64x64 elements each, FP64 multigrid local solves."""
    return deformed_square((8, 8), 3, 64, seed=seed, name="deformed8x8_p3_n64", local_solver="mg",
                           mg_precision=64, primal="vertices+edges",
                           description="2D Poisson on the deformed square, 8x8 patches, p=3, 64^2 elements, "
                                       "FP64 MG V(2,2) Chebyshev local solves, primal vertices + edge averages")


def deformed_16x16_mixed(seed: int = 0) -> Workload:
    """Deformed square, 16x16 patches of uneven size and degree, FP32 multigrid.

    Draw order from ``default_rng(seed)``: xi ~ U(0.5, 1); then for direction
    0 and then direction 1: elements per patch column (row) from
    {32, 48, 64, 96}, 16 draws; degree per patch column (row) from {2, 3, 4},
    16 draws.  Drawing per column/row keeps every shared side conforming.
    """
    rng = np.random.default_rng(seed)
    xi = float(rng.uniform(0.5, 1.0))
    nel, deg = [], []
    for _ in range(2):
        nel.append([int(v) for v in rng.choice([32, 48, 64, 96], size=16)])
        deg.append([int(v) for v in rng.choice([2, 3, 4], size=16)])
    wl = deformed_square((16, 16), deg, nel, amp_factor=xi, name="deformed16x16_mixed", local_solver="mg",
                         mg_precision=32, primal="vertices+edges",
                         description="2D Poisson on the deformed square, 16x16 patches, per-column/per-row "
                                     "elements in {32,48,64,96} and degree in {2,3,4}, FP32 MG")
    wl.seed = seed
    return wl


def cube_4x4x4() -> Workload:
    """Unit cube, 4x4x4 identity patches, p=2, 24^3 elements each, vertices + edge averages, FP32 MG."""
    return unit_cube((4, 4, 4), 2, 24, name="cube4x4x4_p2_n24", local_solver="mg", mg_precision=32,
                     primal="vertices+edges",
                     description="3D Poisson on the unit cube, 4x4x4 affine patches, p=2, 24^3 elements, "
                                 "primal vertices + edge averages, FP32 MG")


def serving_stream(seed: int = 0, n_requests: int = 512,
                   grids=(2, 4, 8), degrees=(2, 3, 4), n_els=(16, 32, 64, 128)) -> List[Request]:
    """Stream of 2D deformed-square solves with random size and sine-series f.

    Per request, in this order from ``default_rng(seed)``: patch grid side
    from ``grids``, degree from ``degrees``, elements per patch direction from
    ``n_els``, xi ~ U(0.5, 1), 3x3 coefficients ~ N(0, 1), then the
    exponential inter-arrival gap (unit rate; scale by 1/rate).
    """
    rng = np.random.default_rng(seed)
    out = []
    t = 0.0
    for i in range(n_requests):
        g = int(rng.choice(grids))
        p = int(rng.choice(degrees))
        n = int(rng.choice(n_els))
        xi = float(rng.uniform(0.5, 1.0))
        coef = rng.standard_normal((3, 3))
        t += float(rng.exponential(1.0))
        f, u = sine_series_rhs(coef)
        wl = deformed_square((g, g), p, n, amp_factor=xi, name=f"req{i}_g{g}_p{p}_n{n}", local_solver="mg",
                             mg_precision=32, primal="vertices+edges")
        wl.f, wl.u_exact = f, u
        wl.extra["coef"] = coef
        out.append(Request(index=i, arrival_unit=t, workload=wl))
    return out


def sub_block(wl: Workload, origin: Sequence[int], size: Sequence[int]) -> Workload:
    """The patches of a rectangular block of ``wl``'s patch grid as a workload of their own
    (same geometry, degrees, knots and f; the block's outer sides become its boundary).
    ``origin`` and ``size`` count patches per direction."""
    idx = []
    ranges = [range(origin[d], origin[d] + size[d]) for d in range(wl.dim)]
    for k in range(int(np.prod(size))):
        pos, r = [], k
        for d in range(wl.dim):
            pos.append(ranges[d][r % size[d]])
            r //= size[d]
        flat, stride = 0, 1
        for d in range(wl.dim):
            flat += pos[d] * stride
            stride *= wl.grid[d]
        idx.append(flat)
    per = [list(wl.extra["dofs_per_dir"][d][origin[d]:origin[d] + size[d]]) for d in range(wl.dim)]
    return Workload(name=f"{wl.name}_block{'_'.join(map(str, origin))}", dim=wl.dim, grid=tuple(size),
                    patches=[wl.patches[i] for i in idx], f=wl.f, u_exact=wl.u_exact,
                    local_solver=wl.local_solver, mg_precision=wl.mg_precision, primal=wl.primal, tol=wl.tol,
                    inner_tol=wl.inner_tol, seed=wl.seed, extra=dict(wl.extra, dofs_per_dir=per))


CONFIGS = {
    "square2x2_p2_n16": square_2x2,
    "deformed8x8_p3_n64": deformed_8x8,
    "deformed16x16_mixed": deformed_16x16_mixed,
    "cube4x4x4_p2_n24": cube_4x4x4,
}
