"""Writes the full-size golden files: the oracle's solution of each benchmark
configuration, sampled at 2000 seeded global coefficients, plus its l2 norm.
Calls only the oracle: the global conforming system with SuperLU for the 2D
configurations; for the 3D cube, where a global sparse LU of ~1M unknowns does
not fit, the oracle's exact-local IETI-DP run to a dual residual of 1e-13 (its
agreement with the global direct solve is pinned by the oracle tests on
smaller cubes).

    python tests/golden/make_golden.py deformed8x8_p3_n64 [deformed16x16_mixed cube4x4x4_p2_n24 ...]
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import conforming, ietidp  # noqa: E402


def make(name: str, nsample: int = 2000):
    wl = W.CONFIGS[name]()
    t0 = time.time()
    if wl.dim == 2:
        u, lay, _ = conforming.solve_direct(wl)
        method = "oracle global conforming system, SuperLU (oracle/conforming.py: solve_direct)"
    else:
        ie = ietidp.IetiDP(wl)
        parts, lam, info = ie.solve(tol=1e-13)
        lay = ie.lay
        u = conforming.global_from_torn(lay, parts)
        method = (f"oracle exact-local IETI-DP (oracle/ietidp.py), CG to 1e-13 in {info['iterations']} "
                  f"iterations")
    free = np.flatnonzero(~lay.boundary)
    rng = np.random.default_rng(12345)
    idx = np.sort(rng.choice(free, size=min(nsample, len(free)), replace=False))
    out = {
        "config": name,
        "method": method,
        "ndof_global": int(len(free)),
        "norm2": float(np.linalg.norm(u)),
        "indices": [int(i) for i in idx],
        "values": [float(v) for v in u[idx]],
        "seconds": round(time.time() - t0, 1),
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"full_{name}.json")
    with open(path, "w") as fh:
        json.dump(out, fh)
    print(f"{name}: {len(free)} dofs, |u| = {out['norm2']:.12e}, {out['seconds']} s -> {path}", flush=True)


if __name__ == "__main__":
    for n in sys.argv[1:]:
        make(n)
