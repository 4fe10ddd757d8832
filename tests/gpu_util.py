"""Helpers for the GPU parity tests: run the HIP solver and the oracle on the same workload."""
import numpy as np

import workloads as W
from oracle import conforming


def split_torn(wl, u):
    parts, off = [], 0
    for p in wl.patches:
        parts.append(np.asarray(u[off:off + p.ndof]))
        off += p.ndof
    return parts


def run_gpu(wl, **opt):
    import torch
    from paper_1705_04531_amd import Solver, options_for
    print(f"[gpu] {wl.name} ndof={wl.ndof_torn} opts={opt}", flush=True)
    s = Solver(wl.patches, options_for(wl, **opt))
    x = s.quadrature(device=False)
    f = torch.from_numpy(wl.f(x)).to("cuda")
    u, st = s.solve(f)
    torch.cuda.synchronize()
    out = u.cpu().numpy()
    s.close()
    return out, st


def oracle_solution(wl):
    u, lay, systems = conforming.solve_direct(wl)
    return u, lay, systems


def rel_err(wl, u_torn, u_ref, lay):
    ug = conforming.global_from_torn(lay, split_torn(wl, u_torn))
    return float(np.linalg.norm(ug - u_ref) / np.linalg.norm(u_ref))


def with_sine_rhs(wl, seed=1):
    rng = np.random.default_rng(seed)
    if wl.dim == 2:
        f, u = W.sine_series_rhs(rng.standard_normal((3, 3)))
    else:
        c = rng.standard_normal(3)

        def f(x, c=c):
            out = np.zeros(x.shape[0])
            for a in range(3):
                out += c[a] * (1 + 2 * a ** 2) * np.pi ** 2 * np.sin((a + 1) * np.pi * x[:, 0]) * \
                    np.sin(np.pi * x[:, 1]) * np.sin((a % 2 + 1) * np.pi * x[:, 2])
            return out
        u = None
    wl.f, wl.u_exact = f, u
    return wl


def golden_errors(golden, u_torn):
    """A torn GPU result against a full-size golden file: relative l2 over the sampled
    coefficients (64 per patch plus 2000 global ones) and the largest sampled deviation over
    the oracle's max norm.  Each sample is read at one torn copy of its coefficient (the
    copies of a returned solution are identical)."""
    idx = np.asarray(golden["torn_positions"])
    ref = np.asarray(golden["values"])
    got = np.asarray(u_torn)[idx]
    l2 = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    linf = float(np.abs(got - ref).max() / golden["max_abs"])
    return l2, linf
