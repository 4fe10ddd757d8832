"""Degenerate and ragged cases on the GPU against the oracle: a single patch (no interface, no
multipliers, no primal unknowns), a zero load, a ragged multigrid hierarchy (patches whose odd element
counts stop the coarsening at the finest level next to patches with three levels), degree-1 patches;
and the untuned smoother choice per dimension and spline degree."""
import numpy as np
import pytest

import workloads as W
from gpu_util import oracle_solution, rel_err, run_gpu, with_sine_rhs

pytestmark = pytest.mark.gpu

VARIANTS = [("mg", {}), ("exact_mg", {"local_solver": 2}), ("mg_saddle", {"local_solver": 3}),
            ("tensor", {"smoother": 1})]
CASES = [
    ("single_patch", lambda: with_sine_rhs(W.deformed_square((1, 1), 3, 16, seed=0, name="single"), 2)),
    ("ragged_levels", lambda: with_sine_rhs(W.deformed_square((2, 2), 2, [[7, 16], [16, 9]], seed=0,
                                                              name="ragged"), 3)),
    ("degree1", lambda: with_sine_rhs(W.deformed_square((2, 2), 1, 16, seed=0, name="p1"), 4)),
    ("single_cube", lambda: W.unit_cube((1, 1, 1), 2, 6, name="single_cube")),
]


@pytest.mark.parametrize("variant,opts", VARIANTS, ids=[v[0] for v in VARIANTS])
@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_edge_case_matches_oracle(require_gpu, name, make, variant, opts):
    wl = make()
    u_ref, lay, _ = oracle_solution(wl)
    u, st = run_gpu(wl, tol=1e-10, coarse_dofs=0, **opts)
    err = rel_err(wl, u, u_ref, lay)
    print(f"{name} {variant}: err={err:.3e} outer={st['outer_iterations']} n_lambda={st['n_lambda']}", flush=True)
    assert np.all(np.isfinite(u))
    assert err <= 1e-8


@pytest.mark.parametrize("variant,opts", VARIANTS, ids=[v[0] for v in VARIANTS])
def test_zero_load_gives_zero(require_gpu, variant, opts):
    wl = W.deformed_square((2, 2), 2, 16, seed=0, name="zero_load")
    wl.f = lambda x: np.zeros(x.shape[0])
    u, st = run_gpu(wl, coarse_dofs=0, **opts)
    print(f"zero load {variant}: max|u|={np.abs(u).max():.3e} breakdown={st['breakdown']}", flush=True)
    assert np.all(np.isfinite(u)) and np.abs(u).max() == 0.0


TABLE_CASES = [
    ("2d_p2", lambda: with_sine_rhs(W.deformed_square((2, 2), 2, 16, seed=0, name="t2p2"), 5), 3),
    ("3d_p2", lambda: W.unit_cube((2, 2, 1), 2, 6, name="t3p2"), 4),
    ("2d_p3", lambda: with_sine_rhs(W.deformed_square((2, 2), 3, 16, seed=0, name="t2p3"), 5), 6),
    ("2d_p4", lambda: with_sine_rhs(W.deformed_square((2, 2), 4, 16, seed=0, name="t2p4"), 5), 7),
    ("2d_p5", lambda: with_sine_rhs(W.deformed_square((2, 2), 5, 16, seed=0, name="t2p5"), 5), 8),
]


@pytest.mark.parametrize("name,make,degree", TABLE_CASES, ids=[c[0] for c in TABLE_CASES])
def test_smoother_table_by_dimension_and_degree(require_gpu, name, make, degree):
    """The Chebyshev degree the library picks without autotuning follows its table by dimension and
    highest spline degree (3D p = 2 takes a higher degree than 2D p = 2), and the solve stays exact."""
    wl = make()
    u_ref, lay, _ = oracle_solution(wl)
    u, st = run_gpu(wl, tol=1e-10, coarse_dofs=0)
    err = rel_err(wl, u, u_ref, lay)
    print(f"{name}: degree {st['cheb_degree']}/{st['cheb_degree_coarse']} err={err:.3e}", flush=True)
    assert st["cheb_degree"] == degree and st["cheb_degree_coarse"] == 2
    assert err <= 1e-8
