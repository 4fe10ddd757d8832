"""ieti_solve_noalloc (scratch in the library's static per-GPU array) against ieti_solve through the
C ABI: the same kernels on the same inputs give bitwise the same solution and statistics, on two calls
in a row, the second on a smaller problem (the array then holds the first call's contents), and the
no-allocation call leaves the handle's own ieti_solve unchanged afterwards."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

KEYS = ("outer_iterations", "inner_iterations_max", "inner_iterations_mean", "residual_final",
        "global_residual", "inner_unconverged", "inner_nonfinite")


def _pair(wl, **opt):
    import torch
    from paper_1705_04531_amd import Solver, options_for
    print(f"[no-alloc] {wl.name} ndof={wl.ndof_torn} opts={opt}", flush=True)
    s = Solver(wl.patches, options_for(wl, **opt))
    x = s.quadrature(device=False)
    f = torch.from_numpy(wl.f(x)).to("cuda")
    u_ref, st_ref = s.solve(f)
    u_na, st_na = s.solve(f, no_alloc=True)
    u_again, st_again = s.solve(f)
    torch.cuda.synchronize()
    out = (u_ref.cpu().numpy(), st_ref, u_na.cpu().numpy(), st_na, u_again.cpu().numpy())
    s.close()
    return out


@pytest.mark.parametrize("variant", ["mg64", "mg32_saddle"])
def test_noalloc_matches_solve_two_calls(require_gpu, variant):
    from paper_1705_04531_amd import _abi
    opt = {"mg_precision": 64} if variant == "mg64" else {"mg_precision": 32,
                                                           "local_solver": _abi.IETI_LOCAL_MG_SADDLE}
    big = W.deformed_square((4, 4), 3, 24, seed=0, name="deformed4x4_p3_n24")
    small = W.deformed_square((2, 2), 2, 12, seed=1, name="deformed2x2_p2_n12")
    for wl in (big, small):   # the second call runs on a smaller input
        u_ref, st_ref, u_na, st_na, u_again = _pair(wl, coarse_dofs=0, tol=1e-10, **opt)
        assert np.array_equal(u_ref, u_na), np.abs(u_ref - u_na).max()
        assert np.array_equal(u_ref, u_again)
        for k in KEYS:
            assert st_ref[k] == st_na[k], (k, st_ref[k], st_na[k])
        assert st_ref["outer_iterations"] > 0
