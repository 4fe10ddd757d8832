"""Serving: each result is the same alone and in the mix (requests of a batch share every launch and the
primal coarse solve, so the same means: within 1e-8 relative l2, the configurations' tolerance, with the
smoother degree fixed by the options), every result matches the oracle, admission by HBM budget."""
import numpy as np
import pytest

import workloads as W
from gpu_util import oracle_solution, rel_err

pytestmark = pytest.mark.gpu


def _small_requests(n=8):
    reqs = [r for r in W.serving_stream(seed=0, n_requests=200) if r.workload.ndof_torn <= 30000]
    return [r.workload for r in reqs[:n]]


def _run(server, wls):
    from paper_1705_04531_amd import quadrature_points
    # loads first, then the submissions back to back, so that requests queue up behind a running batch
    loads = [wl.f(quadrature_points(wl.patches)) for wl in wls]
    tickets = [server.submit(wl.patches, f) for wl, f in zip(wls, loads)]
    out = []
    for t in tickets:
        rc, u, st, times = server.poll(t, wait=True)
        assert rc == 0, rc
        out.append((u, st, times))
    return out


# smoother degrees fixed, so that a request's multigrid does not depend on the highest degree of its batch
FIXED = dict(cheb_degree=6, cheb_degree_coarse=2)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_alone_equals_mix_and_oracle(require_gpu):
    from paper_1705_04531_amd import Server, options_for
    wls = _small_requests(8)
    assert len(wls) == 8
    alone = []
    s1 = Server(options_for(wls[0], batch_dofs=0, **FIXED), slots=1)
    for wl in wls:
        (u, st, _), = _run(s1, [wl])
        alone.append(u)
    s1.close()
    s4 = Server(options_for(wls[0], **FIXED), slots=4)
    res = _run(s4, wls)
    s4.close()
    admits = [times[1] for _, _, times in res]
    print(f"[gpu] serving mix: {len(set(admits))} admissions for {len(wls)} requests", flush=True)
    for wl, a, (u, st, times) in zip(wls, alone, res):
        d = _rel(u, a)
        print(f"{wl.name}: alone vs mix rel diff {d:.2e}", flush=True)
        assert d <= 1e-8
    # every request of the mix is correct
    for wl, (u, st, times) in zip(wls, res):
        u_ref, lay, _ = oracle_solution(wl)
        err = rel_err(wl, u, u_ref, lay)
        print(f"{wl.name}: err={err:.2e} outer={st['outer_iterations']} latency={times[2] - times[0]:.1f} ms",
              flush=True)
        assert err <= 1e-8
        assert times[0] <= times[1] <= times[2]


def test_admission_by_budget(require_gpu):
    from paper_1705_04531_amd import Server, _abi, options_for, quadrature_points
    wls = _small_requests(3)
    # a budget below any request's footprint: refused, not run
    tiny = Server(options_for(wls[0], hbm_budget=1 << 20), slots=2)
    x = quadrature_points(wls[0].patches)
    t = tiny.submit(wls[0].patches, wls[0].f(x))
    rc, _, _, _ = tiny.poll(t, wait=True)
    assert rc == _abi.IETI_ENOMEM
    tiny.close()
    # three identical requests and a budget of 1.5 footprints: all finish, admissions serialised
    from paper_1705_04531_amd import Plan
    need = Plan(wls[0].patches, options_for(wls[0])).device_bytes()
    one = Server(options_for(wls[0], hbm_budget=int(1.5 * need)), slots=3)
    res = _run(one, [wls[0]] * 3)
    one.close()
    spans = sorted((times[1], times[2]) for _, _, times in res)
    for (a0, d0), (a1, d1) in zip(spans, spans[1:]):
        assert a1 >= d0 - 1e-6, "two requests were admitted together under a one-request budget"


def test_batch_with_a_full_size_request(require_gpu):
    """A request of the serving stream with 8x8 patches of 64^2 elements (the largest grid, the benchmark
    patch size) batched with small ones: its result alone and in the batch agree within 1e-8, the small
    ones too, and the batch shares one admission."""
    from paper_1705_04531_amd import Server, options_for
    stream = W.serving_stream(seed=0, n_requests=200)
    big = next(r.workload for r in stream if r.workload.grid == (8, 8) and r.workload.patches[0].n_el[0] == 64)
    small = _small_requests(3)
    wls = [small[0], big, small[1], small[2]]
    print(f"[gpu] batch with {big.name} ndof={big.ndof_torn}", flush=True)
    s1 = Server(options_for(big, batch_dofs=0, **FIXED), slots=1)
    alone = [_run(s1, [wl])[0][0] for wl in wls]
    s1.close()
    # one slot and a queue filled before the worker can take it: the requests behind the first form a batch
    sb = Server(options_for(big, **FIXED), slots=1)
    res = _run(sb, wls)
    sb.close()
    admits = [times[1] for _, _, times in res]
    assert len(set(admits)) < len(wls), "no two requests were batched"
    for wl, a, (u, st, times) in zip(wls, alone, res):
        d = _rel(u, a)
        print(f"{wl.name}: alone vs batch rel diff {d:.2e}, outer {st['outer_iterations']}", flush=True)
        assert d <= 1e-8
