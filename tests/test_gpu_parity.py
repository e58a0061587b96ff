"""GPU parity: the HIP solver against the CPU oracle, element by element.

Every case runs through the C ABI (ctypes binding); int32 results must match
the oracle's (E*, lowest index) exactly.
"""
import json
import os

import numpy as np
import pytest

from conftest import GOLDEN, check_fp32
from paper_2607_04857_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def q():
    import paper_2607_04857_amd as q
    q.lib()
    return q


def _check(q, orc, Q, **kw):
    got = q.solve(Q, **kw)
    exp = orc.solve(Q, k=1)[0]
    print(f"n={Q.shape[0]} {kw} got=({got.energy_i},{got.index}) exp={exp} tier={got.tier}",
          flush=True)
    assert (got.energy_i, got.index) == exp
    return got


@pytest.mark.parametrize("n", list(range(1, 15)))
def test_direct_path(q, orc, n):
    got = _check(q, orc, inputs.uniform_int(n, -100, 100, 1000 + n))
    assert got.tier == 0


TIERS = [1, 2]


@pytest.mark.parametrize("tier", TIERS)
@pytest.mark.parametrize("n", [15, 16, 17, 19, 22])
def test_walk_small(q, orc, n, tier):
    got = _check(q, orc, inputs.uniform_int(n, -1000, 1000, 2000 + n), tier=tier)
    assert got.tier == tier and got.A + got.B == n


@pytest.mark.parametrize("tier", TIERS)
@pytest.mark.parametrize("B", [6, 7, 8, 9, 10])
@pytest.mark.parametrize("L", [6, 7, 0])
def test_split_invariance(q, orc, B, L, tier):
    Q = inputs.uniform_int(21, -500, 500, 77)
    _check(q, orc, Q, B=B, L=L, tier=tier)


@pytest.mark.parametrize("tier", TIERS)
@pytest.mark.parametrize("B,G", [(9, 8), (10, 8), (10, 6), (10, 5), (10, 4), (10, 3)])
@pytest.mark.parametrize("L", [6, 9])
def test_vgpr_levels(q, orc, B, G, L, tier):
    Q = inputs.uniform_int(23, -500, 500, 78)
    got = _check(q, orc, Q, B=B, L=L, tier=tier, vgpr_levels=G)
    assert got.vgpr_levels == G


@pytest.mark.parametrize("tier", TIERS)
def test_ties_zero_matrix(q, orc, tier):
    for n in (15, 18):
        _check(q, orc, np.zeros((n, n), dtype=np.int32), tier=tier)


@pytest.mark.parametrize("tier", TIERS)
def test_ties_diagonal(q, orc, tier):
    rng = np.random.default_rng(5)
    d = rng.integers(-3, 3, size=19, endpoint=True)
    d[::4] = 0
    _check(q, orc, np.diag(d).astype(np.int32), tier=tier)


@pytest.mark.parametrize("tier", TIERS)
def test_all_negative(q, orc, tier):
    _check(q, orc, np.full((17, 17), -1, dtype=np.int32), tier=tier)


@pytest.mark.parametrize("tier", TIERS)
def test_fold_full_matrix(q, orc, tier):
    _check(q, orc, inputs.full_int(18, -300, 300, 9), tier=tier)


@pytest.mark.parametrize("tier", TIERS)
def test_fp32(q, orc, tier):
    for n, seed in ((16, 1), (20, 2)):
        Q = inputs.normal_fp32(n, seed)
        got = q.solve(Q, tier=tier)
        E, idx = orc.solve(Q, k=1)[0]
        check_fp32(orc, Q, got, E, idx)


def _golden():
    with open(os.path.join(GOLDEN, "oracle_results.json")) as f:
        return json.load(f)


@pytest.mark.parametrize("name", ["n24_int_u100_s1", "n30_int_u1000_s10", "n31_int_u10000_s11",
                                  "n33_int_u100_s12", "n36_int_u1000_s2", "n36_planted_u1000_s3",
                                  "n28_fp32_s6", "n32_fp32_s13"])
@pytest.mark.parametrize("tier", TIERS)
def test_stored_oracle_results(q, orc, name, tier):
    g = _golden()
    if name not in g:
        pytest.skip("stored value not generated")
    e = g[name]
    Q = getattr(inputs, e["generator"])(**e["kwargs"])
    if e["generator"] == "planted":
        Q = Q[0]
    got = q.solve(Q, tier=tier)
    print(name, got.energy_i, got.energy, got.index, e["best"], f"{got.kernel_ms:.2f} ms",
          flush=True)
    if e["dtype"] == "int32":
        assert [got.energy_i, got.index] == e["best"]
    else:
        E, idx = e["best"]
        check_fp32(orc, Q, got, E, idx)


@pytest.mark.parametrize("tier", TIERS)
def test_headline_instance_equals_oracle(q, tier):
    """The n = 44 instance of the headline measurement (int32 U[-10^4, 10^4],
    seed 4), solved whole in the default plan, equals the oracle's stored
    answer over all 2^44 states (O2 in resumable shards, written by
    make_oracle_goldens.py)."""
    e = _golden()["n44_int_u10000_s4"]
    assert e["method"] == "O2" and e["kwargs"] == dict(n=44, lo=-10000, hi=10000, seed=4)
    Q = inputs.uniform_int(**e["kwargs"])
    got = q.solve(Q, tier=tier)
    print("headline44", tier, got.energy_i, got.index, e["best"], f"{got.kernel_ms:.1f} ms",
          flush=True)
    assert got.states == 2 ** 44
    assert [got.energy_i, got.index] == e["best"]


@pytest.mark.parametrize("tier", TIERS)
def test_planted_n44(q, orc, tier):
    Q, xstar = inputs.planted(44, -10000, 10000, 8)
    got = q.solve(Q, tier=tier)
    istar = orc.index_of(xstar)
    print("planted44", got.energy_i, got.index, istar, f"{got.kernel_ms:.1f} ms", flush=True)
    assert got.index == istar
    assert got.energy_i == orc.energy(Q, istar)


def test_planted_n48_large(q, orc):
    """Beyond the headline size: 2^48 states (about 5 s), entries U[-1000, 1000]
    with a planted unique ground state, and its top-4 head."""
    Q, xstar = inputs.planted(48, -1000, 1000, 9)
    istar = orc.index_of(xstar)
    got = q.solve(Q)
    print("planted48", got.energy_i, got.index, istar, f"{got.kernel_ms:.1f} ms", flush=True)
    assert (got.A, got.B) == (38, 10)
    assert got.index == istar and got.energy_i == orc.energy(Q, istar)
    res, pairs = q.solve(Q, k=4)
    assert pairs[0] == (got.energy_i, istar)
    # planted: E(x) >= E(x*) + Hamming(x, x*), so every other state is at least one higher
    assert all(e >= got.energy_i + 1 for e, _ in pairs[1:])
    assert all(e == orc.energy(Q, i) for e, i in pairs)
    assert pairs == sorted(pairs)


def _gray(c):
    return c ^ (c >> 1)


def test_headline_sampled_items(q, orc):
    """The n = 44 headline instance in its own plan and kernel, checked on
    sampled work items: item c covers the contiguous index range
    [g(c) 2^(L+B), (g(c)+1) 2^(L+B)) of 2^26 states, which the oracle
    evaluates exhaustively: the first and last pairs of items and ten random
    pairs (2^31 states in all)."""
    Q = inputs.uniform_int(44, -10000, 10000, 4)
    info = q.plan_info(Q)
    L, B, items = info["L"], info["B"], info["items"]
    assert (info["A"], B, L, items) == (34, 10, 16, 1 << 18)
    span = 1 << (L + B)
    rng = np.random.default_rng(44)
    firsts = [0, items - 2] + [int(c) for c in rng.integers(0, items - 2, 10)]
    for c0 in firsts:
        got = q.solve(Q, item_first=c0, item_count=2)
        exp = min(orc.solve_range(Q, _gray(c) * span, span, k=1)[0] for c in range(c0, c0 + 2))
        print(f"items [{c0}, {c0 + 2}): {got.energy_i} @ {got.index} (oracle {exp})", flush=True)
        assert (got.energy_i, got.index) == exp
    c0 = firsts[-1]
    res, pairs = q.solve(Q, k=16, item_first=c0, item_count=1)
    assert pairs == [(int(e), int(i)) for e, i in orc.solve_range(Q, _gray(c0) * span, span, k=16)]


def _gray_inverse(g):
    c = 0
    while g:
        c ^= g
        g >>= 1
    return c


@pytest.mark.parametrize("n,lo", [(54, -1000), (50, -10000)])
def test_large_n_sampled_items(q, orc, n, lo):
    """n = 54 and 50 in their own plans (A = n - 10 prefix bits, the smallest
    items the planner allows: 2^(A-20) Gray steps, one wave each).  A planted
    instance is solved on the work item that holds its ground state, which
    the solve must return, and on a neighbouring item, whose answer must be
    a state of that item's index block with the oracle's energy, above the
    ground state, and with no single flip inside the block improving it (or
    tying it at a lower index)."""
    Q, xstar = inputs.planted(n, lo, -lo, 60 + n)
    istar = orc.index_of(xstar)
    L = n - 10 - 20
    info = q.plan_info(Q, L=L)
    B, items = info["B"], info["items"]
    assert (info["A"], B, info["L"], items) == (n - 10, 10, L, 1 << 20)
    span = 1 << (L + B)
    c = _gray_inverse(istar >> (L + B))
    assert _gray(c) == istar >> (L + B)
    got = q.solve(Q, L=L, item_first=c, item_count=1)
    print(f"n={n} item {c}: {got.energy_i} @ {got.index} (planted {istar}) "
          f"{got.kernel_ms:.1f} ms", flush=True)
    assert got.index == istar and got.energy_i == orc.energy(Q, istar)
    c2 = c + 1 if c + 1 < items else c - 1
    r = q.solve(Q, L=L, item_first=c2, item_count=1)
    base = _gray(c2) * span
    assert base <= r.index < base + span
    assert r.energy_i == orc.energy(Q, r.index) and r.energy_i > got.energy_i
    for b in range(L + B):                                # flips that stay in the block
        j = r.index ^ (1 << b)
        ej = orc.energy(Q, j)
        assert ej > r.energy_i or (ej == r.energy_i and j > r.index), (b, ej)


def test_algebraic_invariances(q, orc):
    """End to end through the walk (n = 26): relabelling the variables
    permutes the argmin, E(cQ) = c E(Q) for an integer c > 0, and the
    maximum of E(Q) is minus the minimum of E(-Q) (checked by the oracle)."""
    n = 26
    Q = inputs.uniform_int(n, -1000, 1000, 2600)
    base = q.solve(Q)
    assert (base.energy_i, base.index) == orc.solve(Q, k=1)[0]
    x = np.array([(base.index >> (n - 1 - i)) & 1 for i in range(n)])
    perm = np.random.default_rng(26).permutation(n)
    Qp = np.ascontiguousarray(Q[np.ix_(perm, perm)])          # variable i' = perm[i]
    rp = q.solve(Qp)
    xp = np.array([(rp.index >> (n - 1 - i)) & 1 for i in range(n)])
    assert rp.energy_i == base.energy_i
    assert orc.energy(Q, orc.index_of(xp[np.argsort(perm)])) == base.energy_i
    if len({e for e, _ in orc.solve(Q, k=2)}) == 2:                # unique minimum
        assert np.array_equal(xp, x[perm])
    r3 = q.solve(3 * Q)
    assert (r3.energy_i, r3.index) == (3 * base.energy_i, base.index)
    rneg = q.solve(-Q)
    worst = orc.solve(-Q, k=1)[0]
    assert (rneg.energy_i, rneg.index) == worst
    assert orc.energy(Q, rneg.index) == -rneg.energy_i


@pytest.mark.parametrize("tier", TIERS)
def test_int32_exactness_edge(q, orc, tier):
    """A dense instance on the int32 exactness limit, sum |T| = 2^30 - 1
    exactly (one more is refused with QUBO_EOVERFLOW): the whole solve, a
    restricted item range (unseeded, so its thresholds start from the
    no-energy value) and top-64, all against the oracle."""
    n = 22
    Q = inputs.edge_int(n, 2**30 - 1, seed=2230)
    info = q.plan_info(Q, tier=tier)
    assert info["sum_abs_t"] == 2**30 - 1
    got = q.solve(Q, tier=tier)
    assert (got.energy_i, got.index) == orc.solve(Q, k=1)[0]
    L, B, items = info["L"], info["B"], info["items"]
    span = 1 << (L + B)
    for c0, cnt in ((0, 1), (items // 3, 2), (items - 1, 1)):
        r = q.solve(Q, tier=tier, item_first=c0, item_count=cnt)
        exp = min(orc.solve_range(Q, _gray(c) * span, span, k=1)[0] for c in range(c0, c0 + cnt))
        assert (r.energy_i, r.index) == exp, (c0, cnt, r, exp)
    res, pairs = q.solve(Q, k=64)
    assert pairs == [(int(e), int(i)) for e, i in orc.solve(Q, k=64)]
    over = Q.copy()
    over[0, 0] += 1 if over[0, 0] >= 0 else -1
    with pytest.raises(q.QuboError) as e:
        q.solve(over)
    assert e.value.status == -2
