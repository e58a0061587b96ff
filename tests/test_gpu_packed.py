"""GPU parity of the packed walk (tier 4: two 16-bit chunk energies per
32-bit word, Sec. IV-B "Data types") against the CPU oracle.

Every int32 result must equal the oracle's (E*, lowest index) exactly.  The
edge cases put the chunk energies at the ends of the 16-bit range: a
suffix-column sum |T| of exactly 32767 with every suffix entry positive
(E_sd reaches +32767), negative (-32767) or mixed, and chunk energies
spanning exactly 65536 values, shifted so that they fill [-32768, 32767].
"""
import json
import os

import numpy as np
import pytest

from conftest import GOLDEN
from paper_2607_04857_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def q():
    import paper_2607_04857_amd as q
    q.lib()
    return q


def _check(q, orc, Q, tier=4, **kw):
    got = q.solve(Q, tier=tier, **kw)
    exp = orc.solve(Q, k=1)[0]
    print(f"n={Q.shape[0]} tier={tier} {kw} got=({got.energy_i},{got.index}) exp={exp} "
          f"plan=(A={got.A},B={got.B},L={got.L},tier={got.tier},G={got.vgpr_levels})", flush=True)
    assert (got.energy_i, got.index) == exp
    assert got.states == 2 ** Q.shape[0]
    return got


@pytest.mark.parametrize("n", [17, 18, 20, 23, 26])
def test_packed_sizes(q, orc, n):
    got = _check(q, orc, inputs.uniform_int(n, -100, 100, 4000 + n))
    assert got.tier == 4 and got.B == 11 and got.A == n - 11


@pytest.mark.parametrize("B,G", [(11, 4), (11, 3), (11, 5), (11, 6), (11, 8), (11, 12),
                                 (10, 8), (10, 12), (9, 12)])
@pytest.mark.parametrize("L", [6, 9, 0])
def test_packed_variants(q, orc, B, G, L):
    Q = inputs.uniform_int(23, -300, 300, 79)
    got = _check(q, orc, Q, B=B, L=L, vgpr_levels=G)
    assert (got.tier, got.B, got.vgpr_levels) == (4, B, G)


@pytest.mark.parametrize("sign", [1, -1, 0])
@pytest.mark.parametrize("n", [19, 24])
def test_packed_16bit_range_edge(q, orc, n, sign):
    """Suffix-column sum 32767: the largest input the packed layout takes;
    with all suffix entries of one sign some chunk energy reaches +-32767."""
    Q = inputs.suffix_edge_int(n, n - 11, 32767, sign, 50 + n + sign)
    got = _check(q, orc, Q)
    assert got.tier == 4


def _suffix_diagonal(n, A, d, seed):
    rng = np.random.default_rng(seed)
    Q = np.triu(rng.integers(-1000, 1000, size=(n, n), endpoint=True)).astype(np.int64)
    Q[:, A:] = 0
    for t, v in enumerate(d):
        Q[A + t, A + t] = v
    return Q.astype(np.int32)


@pytest.mark.parametrize("signs", ["pos", "neg", "mixed"])
def test_packed_shifted_range_edge(q, orc, signs):
    """Only the suffix diagonal is set, with sum |d_t| = 65535: the chunk
    energies span exactly the 16-bit range after the instance's shift, and
    both its ends are reached."""
    n, B = 20, 11
    d = np.full(B, 65535 // B)
    d[0] += 65535 - d.sum()
    if signs == "neg":
        d = -d
    elif signs == "mixed":
        d[1::2] *= -1
    Q = _suffix_diagonal(n, n - B, d, 8)
    info = q.plan_info(Q, tier=4)
    assert info["pack_shift"] == -32768 - int(d[d < 0].sum())
    got = _check(q, orc, Q)
    assert got.tier == 4


@pytest.mark.parametrize("n,R,seed", [(17, 3000, 601), (24, 1000, 5), (28, 1500, 6)])
def test_packed_shifted_random(q, orc, n, R, seed):
    """Entries too large for the suffix-sum bound whose exact chunk-energy
    range still fits 16 bits (the suffix-column sum does not)."""
    Q = inputs.uniform_int(n, -R, R, seed)
    info = q.plan_info(Q, tier=4)
    assert info["pack_shift"] != 0
    got = _check(q, orc, Q)
    assert got.tier == 4


def test_packed_ties(q, orc):
    _check(q, orc, np.zeros((18, 18), dtype=np.int32))
    rng = np.random.default_rng(6)
    d = rng.integers(-3, 3, size=21, endpoint=True)
    d[::3] = 0
    _check(q, orc, np.diag(d).astype(np.int32))
    _check(q, orc, -np.ones((19, 19), dtype=np.int32) * np.tri(19, 19, dtype=np.int32).T)


def _gray(c):
    return c ^ (c >> 1)


def test_packed_item_ranges(q, orc):
    """Restricted item ranges start from no shared best (the thresholds
    start at the no-energy sentinel): each range equals the oracle over its
    contiguous index span."""
    Q = inputs.uniform_int(30, -100, 100, 81)
    info = q.plan_info(Q, tier=4, L=9)
    A, B, L, items = info["A"], info["B"], info["L"], info["items"]
    assert (info["tier"], A, B, L) == (4, 19, 11, 9)
    span = 1 << (L + B)
    for c0 in (0, 7, items - 3):
        got = q.solve(Q, tier=4, L=9, item_first=c0, item_count=3)
        exp = min(orc.solve_range(Q, _gray(c) * span, span, k=1)[0] for c in range(c0, c0 + 3))
        print(f"items [{c0}, {c0 + 3}): {got.energy_i} @ {got.index} (oracle {exp})", flush=True)
        assert (got.energy_i, got.index) == exp


def _golden():
    with open(os.path.join(GOLDEN, "oracle_results.json")) as f:
        return json.load(f)


@pytest.mark.parametrize("name", ["n24_int_u100_s1", "n33_int_u100_s12", "n30_int_u1000_s10",
                                  "n32_int_u1000_s14", "n36_int_u1000_s2"])
def test_packed_stored_oracle_results(q, name):
    """The stored oracle answers of the U[-100, 100] and U[-1000, 1000]
    instances (the n = 24 one is the small single-instance workload, the
    n = 36 one the mid-size one) in the default plan, which packs them (the
    U[-1000, 1000] ones through the exact range), and in forced tier 4."""
    e = _golden()[name]
    Q = getattr(inputs, e["generator"])(**e["kwargs"])
    for kw in ({}, {"tier": 4}):
        got = q.solve(Q, **kw)
        print(name, kw, got.energy_i, got.index, e["best"], got.tier, f"{got.kernel_ms:.3f} ms",
              flush=True)
        assert got.tier == 4
        assert [got.energy_i, got.index] == e["best"]


def test_packed_planted_n40(q, orc):
    """2^40 states with a planted unique ground state, small entries."""
    Q, xstar = inputs.planted(40, -20, 20, 12)
    got = q.solve(Q, tier=4)
    istar = orc.index_of(xstar)
    print("planted40", got.energy_i, got.index, istar, got.tier, f"{got.kernel_ms:.1f} ms",
          flush=True)
    assert got.tier == 4
    assert got.index == istar and got.energy_i == orc.energy(Q, istar)


def test_packed_matches_int32_walk(q):
    """The same instance through tier 4 and tier 2: equal answers (n = 34,
    beyond the oracle's quick range)."""
    Q = inputs.uniform_int(34, -100, 100, 91)
    a = q.solve(Q, tier=4)
    b = q.solve(Q, tier=2)
    print("n34", a.energy_i, a.index, a.kernel_ms, b.energy_i, b.index, b.kernel_ms, flush=True)
    assert a.tier == 4 and b.tier == 2
    assert (a.energy_i, a.index) == (b.energy_i, b.index)


def test_packed_n44_bench_instance(q, orc):
    """The packed bench leg's instance (n = 44, U[-20, 20], seed 4) in its
    default plan (tier 4) and in the int32 walk: the same answer, whose
    energy the oracle confirms and which no single flip improves."""
    Q = inputs.uniform_int(44, -20, 20, 4)
    a = q.solve(Q)
    b = q.solve(Q, tier=2)
    print("n44 packed", a.energy_i, a.index, a.tier, a.B, f"{a.kernel_ms:.1f} ms",
          "int32", b.energy_i, b.index, f"{b.kernel_ms:.1f} ms", flush=True)
    assert a.tier == 4 and a.states == 2 ** 44
    assert (a.energy_i, a.index) == (b.energy_i, b.index)
    assert orc.energy(Q, a.index) == a.energy_i
    for v in range(44):
        assert orc.energy(Q, a.index ^ (1 << v)) >= a.energy_i


def test_packed_n44_sampled_items(q, orc):
    """The packed bench leg's plan (n = 44, entries U[-20, 20]: tier 4,
    B = 11, L = 15, 2^18 items) on sampled work items, each the contiguous
    index range [g(c) 2^(L+B), (g(c)+1) 2^(L+B)) of 2^26 states that the
    oracle evaluates exhaustively: the first and last item pairs and four
    random ones; each range is walked without the shared best (thresholds
    from the no-energy sentinel)."""
    Q = inputs.uniform_int(44, -20, 20, 4)
    info = q.plan_info(Q)
    L, B, items = info["L"], info["B"], info["items"]
    assert (info["tier"], info["A"], B, L, items) == (4, 33, 11, 15, 1 << 18)
    span = 1 << (L + B)
    rng = np.random.default_rng(45)
    firsts = [0, items - 2] + [int(c) for c in rng.integers(0, items - 2, 4)]
    for c0 in firsts:
        got = q.solve(Q, item_first=c0, item_count=2, tier=4, L=L)
        assert (got.tier, got.B, got.L) == (4, B, L)
        exp = min(orc.solve_range(Q, _gray(c) * span, span, k=1)[0] for c in range(c0, c0 + 2))
        print(f"packed items [{c0}, {c0 + 2}): {got.energy_i} @ {got.index} (oracle {exp})",
              flush=True)
        assert (got.energy_i, got.index) == exp


def test_packed_in_batch(q, orc):
    """A batch mixing packable instances (U[-100, 100]) with ones that are
    not (U[-10^4, 10^4]): each result equals the oracle, and the packable
    ones ran tier 4."""
    Qs, lims = [], []
    for i, n in enumerate([18, 20, 21, 22, 24, 19, 23, 20, 22, 24]):
        lims.append((10000, 100, 1000)[i % 3])
        Qs.append(inputs.uniform_int(n, -lims[-1], lims[-1], 600 + i))
    b = q.Batch(Qs)
    for rep in range(2):
        b.run()
        res = b.results()
        for Q, r, lim in zip(Qs, res, lims):
            exp = orc.solve(Q, k=1)[0]
            print(rep, Q.shape[0], lim, r.tier, (r.energy_i, r.index), exp, flush=True)
            assert (r.energy_i, r.index) == exp
            if lim > 1000:
                assert r.tier != 4
        assert any(r.tier == 4 for r in res)
    b.close()


def test_packed_in_server(q, orc):
    """Served requests with entries to 100 (packed by the suffix-column sum),
    to 1000 (packed through the exact range) and to 10^4 (int32 walk),
    submitted together:
    each result equals its lone solve and, for n <= 24, the oracle."""
    Qs, lims = [], []
    for i, n in enumerate([17, 20, 22, 24, 26, 28, 30, 21, 23]):
        lims.append((100, 1000, 10000)[i % 3])
        Qs.append(inputs.uniform_int(n, -lims[-1], lims[-1], 700 + i))
    srv = q.Server(mem_budget_bytes=1 << 30, max_slots=16)
    tickets = [srv.submit(Q) for Q in Qs]
    tiers = []
    for Q, t, lim in zip(Qs, tickets, lims):
        r = srv.wait(t, timeout_ms=60000)
        alone = q.solve(Q)
        print(Q.shape[0], lim, r.tier, alone.tier, (r.energy_i, r.index), flush=True)
        assert (r.energy_i, r.index) == (alone.energy_i, alone.index)
        if Q.shape[0] <= 24:
            assert (r.energy_i, r.index) == orc.solve(Q, k=1)[0]
        if lim <= 100:
            assert r.tier == 4
        if lim > 1000:
            assert r.tier != 4
        tiers.append((lim, r.tier))
    srv.close()
    assert (1000, 4) in tiers            # packed through the exact range


@pytest.mark.parametrize("n,k,R", [(17, 2, 100), (18, 64, 100), (20, 1024, 100), (22, 300, 1000),
                                   (24, 1024, 1000), (26, 512, 100)])
def test_packed_topk(q, orc, n, k, R):
    """Top-k on the packed layout (tier 5): the whole list equals the
    oracle's k smallest (E, index) pairs; R = 1000 packs through the exact
    range."""
    Q = inputs.uniform_int(n, -R, R, 1500 + n)
    res, pairs = q.solve(Q, k=k)
    ref = orc.solve(Q, k=k)
    print(f"packed top-k n={n} k={k} tier {res.tier} B {res.B} "
          f"shift {q.plan_info(Q)['pack_shift']}", flush=True)
    assert res.tier == 5
    assert pairs == [(int(e), int(i)) for e, i in ref]
    assert (res.energy_i, res.index) == pairs[0]


def test_packed_topk_ties_and_forced(q, orc):
    """All-zero and {-1, 0, 1} matrices (ties everywhere) and every packed
    row cache, forced."""
    res, pairs = q.solve(np.zeros((18, 18), dtype=np.int32), k=1024)
    assert res.tier == 5 and pairs == [(0, i) for i in range(1024)]
    rng = np.random.default_rng(78)
    Q = np.triu(rng.integers(-1, 2, (20, 20))).astype(np.int32)
    ref = [(int(e), int(i)) for e, i in orc.solve(Q, k=1024)]
    assert q.solve(Q, k=1024)[1] == ref
    Q = inputs.uniform_int(21, -200, 200, 1601)
    ref = [(int(e), int(i)) for e, i in orc.solve(Q, k=100)]
    for B, G in [(11, 4), (11, 3), (11, 5), (11, 6), (11, 8), (11, 12), (10, 8), (10, 12), (9, 12)]:
        res, pairs = q.solve(Q, k=100, tier=4, B=B, vgpr_levels=G)
        assert (res.tier, res.B, res.vgpr_levels) == (5, B, G)
        assert pairs == ref, (B, G)
