"""GPU batch path: every instance of a mixed batch equals the oracle and its lone solve."""
import numpy as np
import pytest

from conftest import check_fp32
from paper_2607_04857_amd import inputs

pytestmark = pytest.mark.gpu


def _mixed_batch():
    Qs = []
    for k, n in enumerate([3, 9, 14, 15, 16, 18, 20, 21, 15, 19, 22, 17]):
        Qs.append(inputs.uniform_int(n, -100, 100, 300 + k))
    for k, n in enumerate([12, 16, 19]):
        Qs.append(inputs.normal_fp32(n, 400 + k))
    Qs.append(np.zeros((16, 16), dtype=np.int32))
    Qs.append(inputs.planted(20, -50, 50, 7)[0])
    return Qs


@pytest.mark.parametrize("tier", [1, 2])
def test_batch_matches_oracle_and_single(orc, tier):
    import paper_2607_04857_amd as q
    Qs = _mixed_batch()
    b = q.Batch(Qs, tier=tier)
    for rep in range(3):                      # graph replays must agree
        b.run()
        res = b.results()
        for Q, r in zip(Qs, res):
            E, idx = orc.solve(Q, k=1)[0]
            if Q.dtype == np.int32:
                assert (r.energy_i, r.index) == (E, idx), (Q.shape, r, E, idx)
            else:
                check_fp32(orc, Q, r, E, idx)
            alone = q.solve(Q, tier=tier)
            assert (alone.energy_i, alone.index) == (r.energy_i, r.index)
        print(f"tier {tier} replay {rep}: {len(res)} instances ok", flush=True)
    states, ms = b.stats()
    assert states == sum(2.0 ** Q.shape[0] for Q in Qs)
    b.close()


def test_solve_batch_function(orc):
    import paper_2607_04857_amd as q
    Qs = [inputs.uniform_int(n, -1000, 1000, 500 + n) for n in (16, 18, 20)]
    for Q, r in zip(Qs, q.solve_batch(Qs)):
        assert (r.energy_i, r.index) == orc.solve(Q, k=1)[0]


def _flip_check(orc, Q, r):
    """Every single flip of the returned state is no better (and no lower-index tie)."""
    n = Q.shape[0]
    is_int = Q.dtype == np.int32
    E = orc.energy(Q, r.index)
    if is_int:
        assert E == r.energy_i, (n, r, E)
    else:
        assert abs(E - r.energy) <= 1e-9 * float(np.abs(Q.astype(np.float64)).sum()) + 1e-12
    for i in range(n):
        j = r.index ^ (1 << (n - 1 - i))
        Ej = orc.energy(Q, j)
        if is_int:
            assert Ej > E or (Ej == E and j > r.index), (n, i, E, Ej)
        else:
            assert Ej >= r.energy - r.tol, (n, i, r.energy, Ej, r.tol)


@pytest.mark.parametrize("kind,seed", [("int", 5), ("fp32", 6)])
def test_batch_full_config_sampled(orc, kind, seed):
    """The 4096-instance batch (n ~ U{20..34}) exactly as the benchmark replays it.

    Every instance: the returned energy is the oracle's energy of the returned
    state, and no single flip improves it.  A seeded sample of the instances
    the oracle solves in seconds: (E*, index) equal to the oracle's.
    """
    import paper_2607_04857_amd as q
    Qs = inputs.batch(4096, 20, 34, seed=seed, kind=kind)
    b = q.Batch(Qs)
    b.run()
    b.run()
    res = b.results()
    states, _ = b.stats()
    b.close()
    assert states == sum(2.0 ** Q.shape[0] for Q in Qs)
    for Q, r in zip(Qs, res):
        _flip_check(orc, Q, r)
    print(f"{kind}: all {len(Qs)} instances self-consistent and flip-stable", flush=True)
    rng = np.random.default_rng(100 + seed)
    small = [i for i, Q in enumerate(Qs) if Q.shape[0] <= 26]
    big = [i for i, Q in enumerate(Qs) if Q.shape[0] == 29]
    pick = list(rng.choice(small, size=20, replace=False)) + [int(rng.choice(big))]
    for i in pick:
        Q, r = Qs[i], res[i]
        E, idx = orc.solve(Q, k=1)[0]
        if kind == "int":
            assert (r.energy_i, r.index) == (E, idx), (i, Q.shape[0], r, E, idx)
        else:
            check_fp32(orc, Q, r, E, idx)
    print(f"{kind}: {len(pick)} sampled instances equal the oracle", flush=True)
