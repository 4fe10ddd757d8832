"""End-to-end parity of the HIP solver (through the C ABI) with the CPU oracle.

The oracle's global sparse direct solution is the exact discrete solution
that every IETI-DP variant reproduces; the GPU result (copies averaged) must
agree to 1e-8 relative l2.  The torn result must also be continuous."""
import numpy as np
import pytest

import workloads as W
from gpu_util import oracle_solution, rel_err, run_gpu, split_torn, with_sine_rhs
from oracle import conforming

pytestmark = pytest.mark.gpu

CASES_2D = [
    ("square2x2_sine", lambda: with_sine_rhs(W.deformed_square((2, 2), 2, 16, name="square2x2_sine"))),
    ("deformed3x3_mixed", lambda: W.deformed_square((3, 3), [[2, 3, 4], [4, 2, 3]], [[8, 12, 16], [16, 8, 12]],
                                                    amp_factor=0.8, name="deformed3x3_mixed")),
    ("deformed4x4_p3_n24", lambda: with_sine_rhs(W.deformed_square((4, 4), 3, 24, seed=0, name="deformed4x4"), 2)),
    ("deformed3x3_mixed_edges", lambda: W.deformed_square((3, 3), [[2, 3, 4], [4, 2, 3]], [[8, 12, 16], [16, 8, 12]],
                                                          amp_factor=0.8, primal="vertices+edges",
                                                          name="deformed3x3_mixed_edges")),
]
CASES_3D = [
    ("cube2x2x2_n6_sine", lambda: with_sine_rhs(W.unit_cube((2, 2, 2), 2, 6, name="cube2x2x2"))),
    ("cube3x3x2_n6", lambda: W.unit_cube((3, 3, 2), 2, 6, name="cube3x3x2")),
]


@pytest.mark.parametrize("hierarchy", ["default", "full"])
@pytest.mark.parametrize("prec", [64, 32])
@pytest.mark.parametrize("name,make", CASES_2D + CASES_3D, ids=[c[0] for c in CASES_2D + CASES_3D])
def test_solution_matches_oracle(require_gpu, name, make, prec, hierarchy):
    """hierarchy "default": coarsening stops at 512 coefficients (most of these small
    patches are then solved on one level); "full": coarse_dofs = 0 forces the whole
    h-hierarchy, so the V-cycle kernels (smoothing, transfers, fused coarse levels) run."""
    wl = make()
    u_ref, lay, systems = oracle_solution(wl)
    extra = {"coarse_dofs": 0} if hierarchy == "full" else {}
    u, st = run_gpu(wl, mg_precision=prec, tol=1e-10, **extra)
    err = rel_err(wl, u, u_ref, lay)
    parts = split_torn(wl, u)
    # the final FP64 residual ||F - K u|| / ||F|| of the conforming system: the library's value for its own u
    # against the oracle's assembled system applied to the same u (copies averaged on both sides)
    res_o = conforming.global_residual(wl, parts, lay, systems)
    print(f"{name} prec={prec} {hierarchy}: err={err:.3e} outer={st['outer_iterations']} "
          f"inner mean={st['inner_iterations_mean']:.1f} max={st['inner_iterations_max']} "
          f"res={st['global_residual']:.6e} oracle res={res_o:.6e}", flush=True)
    assert err <= 1e-8
    assert st["inner_unconverged"] == 0 and st["inner_nonfinite"] == 0
    # both sides evaluate K u to FP64 rounding: |K||u| / |F| ~ 1e3 here, so they agree to ~1e-13 absolute
    assert abs(st["global_residual"] - res_o) <= 1e-4 * res_o + 1e-12
    # copies of every interface coefficient are identical after averaging
    lo = np.full(lay.nglobal, np.inf)
    hi = np.full(lay.nglobal, -np.inf)
    for g, v in zip(lay.gid, parts):
        np.minimum.at(lo, g, v)
        np.maximum.at(hi, g, v)
    assert np.array_equal(lo, hi)


@pytest.mark.parametrize("name,make", CASES_2D[1:2], ids=[CASES_2D[1][0]])
def test_config_tolerance(require_gpu, name, make):
    """At the configs' outer tolerance 1e-8 the solution error stays at the 1e-8 level."""
    wl = make()
    u_ref, lay, _ = oracle_solution(wl)
    errs = {}
    for tol in (1e-8, 1e-10):
        u, st = run_gpu(wl, mg_precision=32, tol=tol)
        errs[tol] = rel_err(wl, u, u_ref, lay)
        print(f"{name} tol={tol:.0e}: err={errs[tol]:.3e} outer={st['outer_iterations']}", flush=True)
    # the dual residual bounds the solution error only up to a factor ~ cond(M^-1 F); both runs are reported,
    # the configs' tolerance must still give 1e-8 and the tighter one must improve on it
    assert errs[1e-8] <= 1e-8
    assert errs[1e-10] <= 1e-9 and errs[1e-10] <= errs[1e-8]


EXACT_CASES = [
    ("square2x2_p2_n16", lambda: W.square_2x2()),
    ("square2x2_sine_exact", lambda: with_sine_rhs(W.deformed_square((2, 2), 2, 16, name="square2x2_sine"))),
    ("deformed3x3_mixed_edges", CASES_2D[3][1]),
    ("deformed4x4_p3_n24", CASES_2D[2][1]),
]


@pytest.mark.parametrize("name,make", EXACT_CASES, ids=[c[0] for c in EXACT_CASES])
def test_exact_local_matches_oracle(require_gpu, name, make):
    """Exact local solves (banded Cholesky, the D-D form) reproduce the oracle."""
    from paper_1705_04531_amd import _abi
    wl = make()
    u_ref, lay, _ = oracle_solution(wl)
    u, st = run_gpu(wl, local_solver=_abi.IETI_LOCAL_EXACT, tol=1e-10)
    err = rel_err(wl, u, u_ref, lay)
    print(f"{name} exact: err={err:.3e} outer={st['outer_iterations']} breakdown={st['breakdown']}", flush=True)
    assert err <= 1e-9
    assert st["inner_iterations_mean"] == 0


@pytest.mark.parametrize("prec", [64, 32])
@pytest.mark.parametrize("name,make", EXACT_CASES[1:], ids=[c[0] for c in EXACT_CASES[1:]])
def test_exact_neumann_mg_dirichlet_matches_oracle(require_gpu, name, make, prec):
    """D-MG: exact Neumann solves in F with multigrid V-cycles for the Dirichlet
    problems of the preconditioner reproduce the oracle (the preconditioner
    changes only the iteration count)."""
    from paper_1705_04531_amd import _abi
    wl = make()
    u_ref, lay, _ = oracle_solution(wl)
    u, st = run_gpu(wl, local_solver=_abi.IETI_LOCAL_EXACT_MG, mg_precision=prec, tol=1e-10)
    err = rel_err(wl, u, u_ref, lay)
    print(f"{name} D-MG prec={prec}: err={err:.3e} outer={st['outer_iterations']}", flush=True)
    assert err <= 1e-9
    assert st["inner_iterations_mean"] == 0


def test_autotuned_smoother_matches_oracle(require_gpu):
    """The setup-time smoother autotuner changes only the speed: the solution
    still matches the oracle, and the chosen smoother lies in the candidate
    grid around the tuned table."""
    wl = CASES_2D[2][1]()
    u_ref, lay, _ = oracle_solution(wl)
    u0, st0 = run_gpu(wl, tol=1e-10)
    u, st = run_gpu(wl, tol=1e-10, autotune=1)
    err = rel_err(wl, u, u_ref, lay)
    print(f"autotune: err={err:.3e} degree {st0['cheb_degree']}/{st0['cheb_degree_coarse']} -> "
          f"{st['cheb_degree']}/{st['cheb_degree_coarse']} lower x{st['cheb_lower']}", flush=True)
    assert err <= 1e-9
    assert abs(st["cheb_degree"] - st0["cheb_degree"]) <= 1 and st["cheb_degree_coarse"] in (2, 3)
    assert st["cheb_lower"] in (0.67, 1.0, 1.5) and st0["cheb_lower"] == 1.0


@pytest.mark.parametrize("smoother", [0, 1], ids=["chebyshev", "tensor"])
def test_graph_replay_equals_direct_launches(require_gpu, smoother):
    """Flexible-CG iterations replayed from captured HIP graphs (runs of check_every iterations and single
    ones) give bitwise the same result as the same launches sent one by one, over several solves on one
    handle (replays separated by the host's synchronisations and eager work)."""
    import torch
    from paper_1705_04531_amd import Solver, options_for
    wl = W.deformed_square((3, 3), 3, 24, seed=0, name="graph3x3")
    outs = {}
    for g in (0, 1):
        s = Solver(wl.patches, options_for(wl, tol=1e-10, coarse_dofs=0, use_graph=g, smoother=smoother))
        x = s.quadrature(device=False)
        f = torch.from_numpy(wl.f(x)).to("cuda")
        us = []
        for rep in range(3):
            u, st = s.solve(f * (1.0 + rep))
            torch.cuda.synchronize()
            us.append(u.cpu().numpy())
        outs[g] = us
        s.close()
    for a, b in zip(outs[0], outs[1]):
        assert np.array_equal(a, b)
    assert np.allclose(outs[1][2], 3.0 * outs[1][0], rtol=1e-8, atol=0)


def test_solves_reproducible_across_instances(require_gpu):
    """Every solve of a handle, and of a second handle made the same way, gives bitwise the same result, also
    when a handle with another multigrid hierarchy has run before it in the process (the fused coarse kernel
    once lost right-hand-side entries to a late wave's clearing of its LDS, which showed as a one-ulp
    difference in the first solve after such a handle)."""
    import torch
    from paper_1705_04531_amd import Solver, _abi, options_for
    wl = W.deformed_square((4, 4), [[4, 4, 3, 2], [4, 3, 2, 4]], [[48, 32, 24, 16], [32, 48, 16, 24]],
                           amp_factor=0.8, name="repro4x4_mixed")
    def solves(cd, reps):
        s = Solver(wl.patches, options_for(wl, coarse_dofs=cd, smoother=_abi.IETI_SMOOTHER_TENSOR))
        x = s.quadrature(device=False)
        f = torch.from_numpy(wl.f(x)).to("cuda")
        us = []
        for _ in range(reps):
            u, _ = s.solve(f)
            torch.cuda.synchronize()
            us.append(u.cpu().numpy())
        s.close()
        return us
    solves(900, 1)
    a = solves(300, 3)
    b = solves(300, 2)
    for u in a[1:] + b:
        assert np.array_equal(a[0], u)


SADDLE_CASES = [CASES_2D[0], CASES_2D[2], CASES_2D[3], CASES_3D[0]]


@pytest.mark.parametrize("prec", [64, 32])
@pytest.mark.parametrize("name,make", SADDLE_CASES, ids=[c[0] for c in SADDLE_CASES])
def test_saddle_point_bpcg_matches_oracle(require_gpu, name, make, prec):
    """MG-MG-S: Bramble-Pasciak CG on the saddle-point system with V-cycle
    preconditioning of K~ (no inner solves) reaches the oracle's solution.  The
    full h-hierarchy is used so that the V-cycles are real multigrid cycles."""
    from paper_1705_04531_amd import _abi
    wl = make()
    u_ref, lay, _ = oracle_solution(wl)
    u, st = run_gpu(wl, local_solver=_abi.IETI_LOCAL_MG_SADDLE, mg_precision=prec, tol=1e-10, coarse_dofs=0)
    err = rel_err(wl, u, u_ref, lay)
    print(f"{name} MG-MG-S prec={prec}: err={err:.3e} its={st['outer_iterations']} "
          f"res={st['global_residual']:.2e} omega={st['saddle_omega']:.3f} breakdown={st['breakdown']}", flush=True)
    assert err <= 1e-8
    assert st["inner_iterations_mean"] == 0 and st["breakdown"] == 0 and st["saddle_omega"] > 1.0


TENSOR_VARIANTS = [("mg", 0), ("exact_mg", 2), ("mg_saddle", 3)]


@pytest.mark.parametrize("prec", [64, 32])
@pytest.mark.parametrize("variant,solver", TENSOR_VARIANTS, ids=[v[0] for v in TENSOR_VARIANTS])
@pytest.mark.parametrize("name,make", CASES_2D, ids=[c[0] for c in CASES_2D])
def test_tensor_smoother_matches_oracle(require_gpu, name, make, variant, solver, prec):
    """The finest-level tensor smoother (p-robust multigrid, Sec. 4) in every multigrid variant: the
    solution still matches the oracle's direct solution (the full h-hierarchy, so V-cycles are real)."""
    from paper_1705_04531_amd import _abi
    wl = make()
    u_ref, lay, _ = oracle_solution(wl)
    u, st = run_gpu(wl, local_solver=solver, mg_precision=prec, tol=1e-10, coarse_dofs=0,
                    smoother=_abi.IETI_SMOOTHER_TENSOR)
    err = rel_err(wl, u, u_ref, lay)
    print(f"{name} tensor smoother {variant} prec={prec}: err={err:.3e} outer={st['outer_iterations']} "
          f"inner={st['inner_iterations_mean']:.2f}", flush=True)
    assert err <= 1e-8
    assert st["cheb_degree"] == 0


@pytest.mark.parametrize("n1", [132, 260], ids=["fused", "unfused"])
@pytest.mark.parametrize("prec", [64, 32])
def test_tensor_smoother_wide_patches(require_gpu, prec, n1):
    """2D patches with more than 128 coefficients per direction (2x1 deformed square, p = 4, 136 and 128
    elements along x: 140 and 132 coefficients, padded to 144; along y 136 coefficients (the products fused
    in pairs per column block) or 264, padded to 272 (above the fused kernels' limit, the four separate
    products): the tensor smoother has no size limit in 2D, and the solve still matches the oracle."""
    from paper_1705_04531_amd import _abi
    wl = W.deformed_square((2, 1), 4, [[136, 128], [n1]], amp_factor=0.8, name="wide2x1_p4")
    u_ref, lay, _ = oracle_solution(wl)
    u, st = run_gpu(wl, local_solver=0, mg_precision=prec, tol=1e-10, smoother=_abi.IETI_SMOOTHER_TENSOR)
    err = rel_err(wl, u, u_ref, lay)
    print(f"wide2x1_p4 tensor smoother prec={prec}: err={err:.3e} outer={st['outer_iterations']} "
          f"inner={st['inner_iterations_mean']:.2f}", flush=True)
    assert err <= 1e-8
    assert st["cheb_degree"] == 0


def test_tensor_smoother_p_robust(require_gpu):
    """p-robustness (Sec. 4): on the same 2x2 deformed square with 32^2 elements per patch and the
    full h-hierarchy, degrees 2..6, both smoothers reach the oracle's solution; the tensor smoother's
    inner flexible-CG iteration count stays bounded as p grows (the Chebyshev smoother's is reported
    beside it, and the tensor smoother's with degree-1 coarse levels and L2 transfers, the paper's full
    p-robust multigrid)."""
    from paper_1705_04531_amd import _abi
    rows = []
    for p in (2, 3, 4, 5, 6):
        wl = with_sine_rhs(W.deformed_square((2, 2), p, 32, seed=0, name=f"deformed2x2_p{p}"), 3)
        u_ref, lay, _ = oracle_solution(wl)
        its = {}
        for name, sm, cd in (("chebyshev", _abi.IETI_SMOOTHER_CHEBYSHEV, 0), ("tensor", _abi.IETI_SMOOTHER_TENSOR, 0),
                             ("tensor_p1", _abi.IETI_SMOOTHER_TENSOR, 1)):
            u, st = run_gpu(wl, tol=1e-10, coarse_dofs=0, smoother=sm, coarse_degree=cd)
            err = rel_err(wl, u, u_ref, lay)
            assert err <= 1e-8, (p, name, err)
            its[name] = st["inner_iterations_mean"]
        rows.append((p, its["chebyshev"], its["tensor"], its["tensor_p1"]))
        print(f"p={p}: inner iterations Chebyshev {its['chebyshev']:.2f}, tensor {its['tensor']:.2f}, "
              f"tensor with degree-1 coarse levels {its['tensor_p1']:.2f}", flush=True)
    tens = [r[2] for r in rows]
    assert max(tens) <= 16.0 and max(tens) <= 1.6 * min(tens), rows


@pytest.mark.parametrize("prec", [64, 32])
@pytest.mark.parametrize("variant,solver", [("mg", 0), ("mg_saddle", 3)], ids=["mg", "mg_saddle"])
@pytest.mark.parametrize("name,make", CASES_3D, ids=[c[0] for c in CASES_3D])
def test_tensor_smoother_3d_matches_oracle(require_gpu, name, make, variant, solver, prec):
    """The tensor smoother on 3D patches (three axis contractions per transform)."""
    from paper_1705_04531_amd import _abi
    wl = make()
    u_ref, lay, _ = oracle_solution(wl)
    u, st = run_gpu(wl, local_solver=solver, mg_precision=prec, tol=1e-10, coarse_dofs=0,
                    smoother=_abi.IETI_SMOOTHER_TENSOR)
    err = rel_err(wl, u, u_ref, lay)
    print(f"{name} 3D tensor smoother {variant} prec={prec}: err={err:.3e} outer={st['outer_iterations']} "
          f"inner={st['inner_iterations_mean']:.2f}", flush=True)
    assert err <= 1e-8


def test_autotune_cache(require_gpu, tmp_path):
    """The autotuner's choice (smoother degrees, interval, finest-level tile variant) goes to the cache file
    on a miss and comes back from it on the next setup with the same key; both solves match the oracle."""
    wl = CASES_2D[2][1]()
    u_ref, lay, _ = oracle_solution(wl)
    cache = str(tmp_path / "tune.jsonl")
    u1, st1 = run_gpu(wl, tol=1e-10, autotune=1, tune_cache=cache)
    lines = open(cache).read().splitlines()
    assert len(lines) == 1 and '"stage": ' in lines[0]
    u2, st2 = run_gpu(wl, tol=1e-10, autotune=1, tune_cache=cache)
    assert st1["tune_cached"] == 0 and st2["tune_cached"] == 1
    for k in ("cheb_degree", "cheb_degree_coarse", "cheb_lower", "fine_tile_staged"):
        assert st1[k] == st2[k], k
    assert len(open(cache).read().splitlines()) == 1
    for u in (u1, u2):
        assert rel_err(wl, u, u_ref, lay) <= 1e-8
    print(f"autotune cache: {lines[0]}", flush=True)


EDGE_ONLY_CASES = [
    ("cube2x2x2_edges", lambda: with_sine_rhs(W.unit_cube((2, 2, 2), 2, 6, primal="edges", name="cube2x2x2_edges"))),
    ("cube3x3x2_edges", lambda: W.unit_cube((3, 3, 2), 2, 6, primal="edges", name="cube3x3x2_edges")),
    ("cube3x3x3_edges_floating", lambda: with_sine_rhs(W.unit_cube((3, 3, 3), 2, 6, primal="edges",
                                                                   name="cube3x3x3_edges"))),
    ("deformed3x3_sides_only_floating", lambda: W.deformed_square((3, 3), [[2, 3, 4], [4, 2, 3]],
                                                                  [[8, 12, 16], [16, 8, 12]], amp_factor=0.8,
                                                                  primal="edges", name="deformed3x3_sides_only")),
]


@pytest.mark.parametrize("hierarchy", ["default", "full"])
@pytest.mark.parametrize("prec", [64, 32])
@pytest.mark.parametrize("name,make", EDGE_ONLY_CASES, ids=[c[0] for c in EDGE_ONLY_CASES])
def test_edge_only_primal_matches_oracle(require_gpu, name, make, prec, hierarchy):
    """The paper's primal set of Sec. 4 in 3D (edge averages only; in 2D the side averages): vertex copies
    are dual, and the centre patch of the 3x3x3 cube and of the 3x3 square floats (no Dirichlet coefficient),
    so its local problems are the semi-definite ones of eq. (6)/(7) with only the edge constraints fixing the
    constants.  The GPU result equals the oracle's global direct solution, and the primal basis is built to
    basis_tol on the floating patches as on the others."""
    wl = make()
    u_ref, lay, _ = oracle_solution(wl)
    extra = {"coarse_dofs": 0} if hierarchy == "full" else {}
    u, st = run_gpu(wl, mg_precision=prec, tol=1e-10, **extra)
    err = rel_err(wl, u, u_ref, lay)
    print(f"{name} prec={prec} {hierarchy}: err={err:.3e} outer={st['outer_iterations']} n_primal={st['n_primal']} "
          f"n_lambda={st['n_lambda']} inner mean={st['inner_iterations_mean']:.1f} max={st['inner_iterations_max']}",
          flush=True)
    assert err <= 1e-8
    assert st["inner_unconverged"] == 0 and st["inner_nonfinite"] == 0


EXACT_3D = [
    ("cube2x2x2_n6_sine", CASES_3D[0][1]),
    ("cube3x3x2_n6", CASES_3D[1][1]),
    ("cube3x3x2_edges", EDGE_ONLY_CASES[1][1]),
]


@pytest.mark.parametrize("variant", ["exact", "exact_mg64", "exact_mg32"])
@pytest.mark.parametrize("name,make", EXACT_3D, ids=[c[0] for c in EXACT_3D])
def test_exact_local_3d_matches_oracle(require_gpu, name, make, variant):
    """3D exact local solves: the block-band Cholesky factors are built on the device (batched over patches
    and modes) and the solves stream them from HBM; the D-D form and D-MG (exact Neumann, multigrid
    Dirichlet problems) reproduce the oracle."""
    from paper_1705_04531_amd import _abi
    wl = make()
    u_ref, lay, _ = oracle_solution(wl)
    opt = {"local_solver": _abi.IETI_LOCAL_EXACT} if variant == "exact" else \
        {"local_solver": _abi.IETI_LOCAL_EXACT_MG, "mg_precision": int(variant[-2:])}
    u, st = run_gpu(wl, tol=1e-10, **opt)
    err = rel_err(wl, u, u_ref, lay)
    print(f"{name} {variant}: err={err:.3e} outer={st['outer_iterations']}", flush=True)
    assert err <= 1e-9
    assert st["inner_iterations_mean"] == 0


P1_CASES = [
    ("deformed3x3_mixed", CASES_2D[1][1]),
    ("deformed4x4_p3_n24", CASES_2D[2][1]),
    ("cube2x2x2_n6_sine", CASES_3D[0][1]),
    ("deformed3x3_sides_only_floating", EDGE_ONLY_CASES[3][1]),
]


@pytest.mark.parametrize("smoother", ["chebyshev", "tensor"])
@pytest.mark.parametrize("prec", [64, 32])
@pytest.mark.parametrize("name,make", P1_CASES, ids=[c[0] for c in P1_CASES])
def test_degree1_coarse_levels_match_oracle(require_gpu, name, make, prec, smoother):
    """Multigrid with degree 1 on every level but the finest (Sec. 4): non-nested levels joined by the L2
    projection of the parameter domain (M_f^{-1} M_fc, line solves with the 1D mass factors) -- a different
    preconditioner, the same solution."""
    wl = make()
    u_ref, lay, _ = oracle_solution(wl)
    opt = {"smoother": 1} if smoother == "tensor" else {}
    u, st = run_gpu(wl, mg_precision=prec, tol=1e-10, coarse_dofs=0, coarse_degree=1, **opt)
    err = rel_err(wl, u, u_ref, lay)
    print(f"{name} p1-coarse {smoother} prec={prec}: err={err:.3e} outer={st['outer_iterations']} "
          f"inner mean={st['inner_iterations_mean']:.1f} max={st['inner_iterations_max']}", flush=True)
    assert err <= 1e-8
    assert st["inner_unconverged"] == 0 and st["inner_nonfinite"] == 0
