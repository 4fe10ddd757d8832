"""Serving: each result is the same alone and in the mix, admission by HBM budget."""
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
    tickets = []
    for wl in wls:
        x = quadrature_points(wl.patches)
        tickets.append(server.submit(wl.patches, wl.f(x)))
    out = []
    for t in tickets:
        rc, u, st, times = server.poll(t, wait=True)
        assert rc == 0, rc
        out.append((u, st, times))
    return out


def test_alone_equals_mix_and_oracle(require_gpu):
    from paper_1705_04531_amd import Server, options_for
    wls = _small_requests(8)
    assert len(wls) == 8
    target = wls[3]
    print(f"[gpu] serving target {target.name} ndof={target.ndof_torn}", flush=True)
    s1 = Server(options_for(target), slots=1)
    (u_alone, st_alone, _), = _run(s1, [target])
    s1.close()
    s4 = Server(options_for(target), slots=4)
    res = _run(s4, wls)
    s4.close()
    u_mix = res[3][0]
    assert np.array_equal(u_alone, u_mix), np.abs(u_alone - u_mix).max()
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
