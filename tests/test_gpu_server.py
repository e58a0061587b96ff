"""GPU serving path: continuous batching returns, for every request, exactly
the result of solving it alone, within the memory budget."""
import threading
import time

import numpy as np
import pytest

from paper_2607_04857_amd import inputs

pytestmark = pytest.mark.gpu


def _same(a, b):
    return (a.energy_i, a.index, a.p) == (b.energy_i, b.index, b.p)


def test_server_mix_equals_alone_and_oracle(orc):
    import paper_2607_04857_amd as q
    reqs = inputs.poisson_requests(40, rate_hz=400.0, n_lo=10, n_hi=26, seed=17)
    srv = q.Server(mem_budget_bytes=256 << 20, max_slots=64)
    t0 = time.perf_counter()
    tickets = []
    for arrival, Q in reqs:                    # replay the Poisson arrival times
        while time.perf_counter() - t0 < arrival:
            time.sleep(0.0002)
        tickets.append((srv.submit(Q), Q))
    for t, Q in tickets:
        r = srv.wait(t, timeout_ms=60000)
        assert r is not None
        alone = q.solve(Q)
        assert _same(r, alone), (Q.shape, r, alone)
        E, idx = orc.solve(Q, k=1)[0]
        if Q.dtype == np.int32:
            assert (r.energy_i, r.index) == (E, idx)
        else:
            assert abs(r.energy - E) <= r.tol
    st = srv.stats()
    info = srv.info()
    print(st, info, flush=True)
    assert st["p50_ms"] > 0 and st["p99_ms"] >= st["p50_ms"] and st["states_per_s"] > 0
    assert info["mem_in_use"] == 0 and info["ticks"] >= 1
    srv.close()


def test_server_memory_budget_defers_admission(orc):
    import paper_2607_04857_amd as q
    Qs = [inputs.uniform_int(n, -100, 100, 900 + n) for n in (24, 25, 26, 27, 28, 24, 25)]
    budget = 180 * 1024                        # two requests of these sizes at a time
    srv = q.Server(mem_budget_bytes=budget, max_slots=32)
    ts = [srv.submit(Q) for Q in Qs]
    for t, Q in zip(ts, Qs):
        r = srv.wait(t, timeout_ms=60000)
        assert (r.energy_i, r.index) == orc.solve(Q, k=1)[0]
    info = srv.info()
    print(info, flush=True)
    assert 0 < info["mem_peak"] <= budget
    assert info["active_peak"] < len(Qs)       # admission was deferred at least once
    srv.close()


def test_server_concurrent_submitters():
    import paper_2607_04857_amd as q
    srv = q.Server(mem_budget_bytes=64 << 20, max_slots=16)
    results = {}

    def worker(k):
        Q = inputs.uniform_int(15 + k % 8, -1000, 1000, 1200 + k)
        t = srv.submit(Q)
        results[k] = (Q, srv.wait(t, timeout_ms=60000))

    th = [threading.Thread(target=worker, args=(k,)) for k in range(12)]
    for x in th:
        x.start()
    for x in th:
        x.join()
    for k, (Q, r) in results.items():
        alone = q.solve(Q)
        assert _same(r, alone)
    srv.close()


def test_server_errors():
    import paper_2607_04857_amd as q
    srv = q.Server(mem_budget_bytes=1 << 20, max_slots=4)
    with pytest.raises(q.QuboError) as e:
        srv.submit(np.zeros((61, 61), dtype=np.int32))
    assert e.value.status == -1
    big = inputs.uniform_int(40, -10, 10, 1)       # needs more than the 1 MiB budget
    with pytest.raises(q.QuboError) as e:
        srv.submit(big)
    assert e.value.status == -4
    with pytest.raises(q.QuboError):
        srv.poll(987654321)
    t = srv.submit(inputs.uniform_int(12, -5, 5, 2))
    r = srv.wait(t, timeout_ms=60000)
    assert r is not None
    srv.close()
