"""GPU batch path: every instance of a mixed batch equals the oracle and its lone solve."""
import numpy as np
import pytest

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
                assert abs(r.energy - E) <= r.tol
                assert r.index == idx or r.energy <= E + r.tol
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
