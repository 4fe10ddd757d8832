"""Writes the full-size golden files: the oracle's solution of each benchmark
configuration, sampled at 64 seeded coefficients of every patch (interior,
side, edge and vertex coefficients alike, boundary excluded) plus 2000 seeded
global coefficients, with its l2 and max norms, and for each sampled global
coefficient one position in the torn (patch-by-patch) layout that holds a copy
of it, so that a torn GPU result can be compared without the oracle's layout.  Calls only the oracle: the
global conforming system with SuperLU for the 2D configurations; for the 3D
cube, where a global sparse LU of ~1M unknowns does not fit, the oracle's
exact-local IETI-DP run to a dual residual of 1e-13 (its agreement with the
global direct solve is pinned by the oracle tests on smaller cubes).

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

PER_PATCH = 64
GLOBAL = 2000


def sample_indices(lay, seed: int = 12345) -> np.ndarray:
    """Global indices sampled: PER_PATCH per patch among its non-boundary coefficients, then GLOBAL more."""
    rng = np.random.default_rng(seed)
    picks = []
    for g in lay.gid:
        cand = g[~lay.boundary[g]]
        picks.append(rng.choice(cand, size=min(PER_PATCH, len(cand)), replace=False))
    free = np.flatnonzero(~lay.boundary)
    picks.append(rng.choice(free, size=min(GLOBAL, len(free)), replace=False))
    return np.unique(np.concatenate(picks))


def make(name: str):
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
    idx = sample_indices(lay)
    # first torn position of every global coefficient (patches in order, copies identical in a result)
    first = np.full(len(lay.boundary), -1, dtype=np.int64)
    off = 0
    for g in lay.gid:
        new = first[g] < 0
        first[g[new]] = off + np.flatnonzero(new)
        off += len(g)
    torn = first[idx]
    assert (torn >= 0).all()
    out = {
        "config": name,
        "method": method,
        "ndof_global": int(np.count_nonzero(~lay.boundary)),
        "norm2": float(np.linalg.norm(u)),
        "max_abs": float(np.abs(u).max()),
        "per_patch": PER_PATCH,
        "indices": [int(i) for i in idx],
        "values": [float(v) for v in u[idx]],
        "torn_positions": [int(t) for t in torn],
        "seconds": round(time.time() - t0, 1),
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"full_{name}.json")
    with open(path, "w") as fh:
        json.dump(out, fh)
    print(f"{name}: {out['ndof_global']} dofs, {len(idx)} samples, |u| = {out['norm2']:.12e}, "
          f"{out['seconds']} s -> {path}", flush=True)


if __name__ == "__main__":
    for n in sys.argv[1:]:
        make(n)
