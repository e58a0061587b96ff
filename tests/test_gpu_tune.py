"""GPU side of plan tuning: the autotuner's runs, its cache, and batches and
server ticks whose instances run different walk variants (one launch per
variant group)."""
import json

import numpy as np
import pytest

from conftest import check_fp32
from paper_2607_04857_amd import inputs

pytestmark = pytest.mark.gpu

# (B, vgpr_levels, tier): every built walk variant in both tiers, cycled over n
VARIANTS = [(10, 4, 2), (10, 5, 1), (9, 8, 2), (8, 12, 1), (10, 8, 2), (7, 12, 2),
            (10, 12, 1), (6, 12, 2), (9, 12, 1), (10, 6, 1), (10, 5, 2), (9, 8, 1),
            (10, 4, 1), (10, 6, 2), (10, 3, 2), (10, 3, 1)]


@pytest.fixture()
def q():
    import paper_2607_04857_amd as q
    q.tune_clear()
    yield q
    q.tune_clear()


def _table(ns, dtype="int32", scope="batch"):
    return [{"n": n, "dtype": dtype, "B": VARIANTS[k % len(VARIANTS)][0], "L": 0,
             "tier": VARIANTS[k % len(VARIANTS)][2], "vgpr_levels": VARIANTS[k % len(VARIANTS)][1],
             "scope": scope}
            for k, n in enumerate(ns)]


def _check(orc, Q, r):
    E, idx = orc.solve(Q, k=1)[0]
    if Q.dtype == np.int32:
        assert (r.energy_i, r.index) == (E, idx), (Q.shape, r, E, idx)
    else:
        check_fp32(orc, Q, r, E, idx)


def _base(r):
    """(B, tier, vgpr_levels) of the int32 plan a result ran: a packed
    (tier-4) result is its plan one suffix bit wider, so its tier is
    reported as None (the tuned tier is not observable)."""
    return (r.B - 1, None, r.vgpr_levels) if r.tier == 4 else (r.B, r.tier, r.vgpr_levels)


def _same_plan(r, e):
    b = _base(r)
    return (b[0], b[2]) == (e["B"], e["vgpr_levels"]) and b[1] in (None, e["tier"])


def test_autotune_writes_cache_and_drives_solves(q, orc, tmp_path):
    path = str(tmp_path / "tune.json")
    won = q.autotune(20, 22, "int32", reps=1, cache_path=path)
    assert [e["n"] for e in won] == [20, 21, 22]
    key = q.device_key()
    assert key.startswith("gfx")
    doc = json.load(open(path))
    assert doc["device"] == key and len(doc["entries"]) == 3
    q.tune_clear()
    assert q.tune_load(path) == 3
    for e in won:
        assert q.tune_lookup(e["n"]) == e
        Q = inputs.uniform_int(e["n"], -1000, 1000, 40 + e["n"])
        r = q.solve(Q)
        assert _same_plan(r, e)
        _check(orc, Q, r)
        print(f"tuned n={e['n']}: {e}", flush=True)
    # a second run merges into the same file
    q.autotune(23, 23, "fp32", reps=0, cache_path=path)
    doc = json.load(open(path))
    assert sorted((x["n"], x["dtype"]) for x in doc["entries"]) == \
        [(20, "int32"), (21, "int32"), (22, "int32"), (23, "fp32")]


def test_batch_with_mixed_variants(q, orc):
    ns = list(range(16, 28))
    q.tune_set(_table(ns) + _table(ns, "fp32"))
    Qs = [inputs.uniform_int(n, -100, 100, 700 + n) for n in ns]
    Qs += [inputs.normal_fp32(n, 800 + n) for n in (16, 18, 22)]
    Qs += [inputs.uniform_int(n, -100, 100, 720 + n) for n in (3, 26, 20, 21)]
    b = q.Batch(Qs)
    for rep in range(2):
        b.run()
        res = b.results()
        for Q, r in zip(Qs, res):
            n = Q.shape[0]
            if n > 14:
                e = q.tune_lookup(n, "fp32" if Q.dtype == np.float32 else "int32", "batch")
                assert _same_plan(r, e)
            _check(orc, Q, r)
        print(f"mixed-variant batch replay {rep}: {len(res)} ok", flush=True)
    b.close()


def test_server_with_mixed_variants(q, orc):
    ns = list(range(16, 28))
    q.tune_set(_table(ns) + _table(ns, "fp32"))
    Qs = [inputs.uniform_int(n, -100, 100, 760 + n) for n in ns for _ in range(2)]
    Qs += [inputs.normal_fp32(n, 860 + n) for n in (16, 24)]
    srv = q.Server(mem_budget_bytes=1 << 30, max_slots=64)
    tickets = [srv.submit(Q) for Q in Qs]
    for Q, t in zip(Qs, tickets):
        r = srv.wait(t, timeout_ms=60000)
        assert r is not None
        e = q.tune_lookup(Q.shape[0], "fp32" if Q.dtype == np.float32 else "int32", "batch")
        assert _same_plan(r, e)
        _check(orc, Q, r)
    srv.close()
    print(f"mixed-variant server: {len(Qs)} ok", flush=True)


def test_single_scope_entries_do_not_steer_batches(q, orc):
    """A lone-solve entry leaves batch instances on the built-in plan and vice versa."""
    q.tune_set([{"n": 22, "B": 7, "L": 0, "tier": 1, "vgpr_levels": 12, "scope": "single"},
                {"n": 23, "B": 8, "L": 0, "tier": 1, "vgpr_levels": 12, "scope": "batch"}])
    Q22, Q23 = inputs.uniform_int(22, -100, 100, 901), inputs.uniform_int(23, -100, 100, 902)
    lone22, lone23 = q.solve(Q22), q.solve(Q23)
    assert (lone22.B, lone22.tier) == (7, 1)      # no packed variant at B = 7
    assert _base(lone23)[::2] == (10, 4)
    b = q.Batch([Q22, Q23])
    b.run()
    r22, r23 = b.results()
    b.close()
    assert _base(r22)[::2] == (10, 4)
    assert _base(r23)[0] == 8 and _base(r23)[1] in (None, 1)
    for Q, r in ((Q22, r22), (Q23, r23), (Q22, lone22), (Q23, lone23)):
        _check(orc, Q, r)


def test_batch_autotune(q, orc, tmp_path):
    path = str(tmp_path / "tune.json")
    won = q.autotune(20, 21, "int32", reps=0, cache_path=path, batch=True)
    assert [(e["n"], e["scope"], e["L"]) for e in won] == [(20, "batch", 0), (21, "batch", 0)]
    doc = json.load(open(path))
    assert sorted((x["n"], x["scope"]) for x in doc["entries"]) == [(20, "batch"), (21, "batch")]
    q.tune_clear()
    assert q.tune_load(path) == 2
    assert q.tune_lookup(20) is None
    Qs = [inputs.uniform_int(n, -100, 100, 950 + n) for n in (20, 21, 20)]
    b = q.Batch(Qs)
    b.run()
    for Q, r in zip(Qs, b.results()):
        e = q.tune_lookup(Q.shape[0], "int32", "batch")
        assert _same_plan(r, e)
        _check(orc, Q, r)
    b.close()
    print(f"batch-tuned: {won}", flush=True)
