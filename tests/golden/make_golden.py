"""Writes the full-size golden files: the oracle's global direct solution of
each benchmark configuration, sampled at 2000 seeded global coefficients, plus
its l2 norm.  Calls only the oracle (global conforming assembly + SuperLU).

    python tests/golden/make_golden.py deformed8x8_p3_n64 [deformed16x16_mixed ...]
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import conforming  # noqa: E402


def make(name: str, nsample: int = 2000):
    wl = W.CONFIGS[name]()
    t0 = time.time()
    u, lay, _ = conforming.solve_direct(wl)
    free = np.flatnonzero(~lay.boundary)
    rng = np.random.default_rng(12345)
    idx = np.sort(rng.choice(free, size=min(nsample, len(free)), replace=False))
    out = {
        "config": name,
        "method": "oracle global conforming system, SuperLU (oracle/conforming.py: solve_direct)",
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
