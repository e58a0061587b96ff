"""GPU: solving by outer-bit reduction (the 2^k reduced instances as one
batch) gives the same (E, lowest index) as a direct solve and the oracle."""
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


@pytest.mark.parametrize("n,k,seed", [(18, 1, 1), (24, 4, 2), (27, 9, 3)])
def test_equals_direct_and_oracle(q, orc, n, k, seed):
    rng = np.random.default_rng(seed)
    Q = rng.integers(-1000, 1001, (n, n)).astype(np.int32)      # full matrix: folded
    got = q.solve_outer(Q, k)
    direct = q.solve(Q)
    print(f"n={n} k={k} outer ({got.energy_i}, {got.index}) direct ({direct.energy_i}, "
          f"{direct.index})", flush=True)
    assert (got.energy_i, got.index) == (direct.energy_i, direct.index)
    assert (got.energy_i, got.index) == orc.solve(Q, k=1)[0]
    assert got.states == 2 ** n


def test_ties_resolve_to_the_lowest_index(q, orc):
    """Diagonal with zeros: many states tie at the minimum, spread over the
    reduced instances; the lowest index must win across them."""
    Q = np.diag(np.array([0, -3, 0, -1, 0, 0, -2, 0, 0, -5, 0, 0, 0, -1, 0, 0, 0, 0],
                         dtype=np.int32))
    got = q.solve_outer(Q, 5)
    assert (got.energy_i, got.index) == orc.solve(Q, k=1)[0]


def test_stored_oracle_n36(q):
    with open(os.path.join(GOLDEN, "oracle_results.json")) as f:
        e = json.load(f)["n36_int_u1000_s2"]
    Q = inputs.uniform_int(**e["kwargs"])
    got = q.solve_outer(Q, 6)
    assert [got.energy_i, got.index] == e["best"]


def test_planted_n44(q, orc):
    Q, xstar = inputs.planted(44, -10000, 10000, 8)
    got = q.solve_outer(Q, 8)
    istar = orc.index_of(xstar)
    print("outer planted44", got.energy_i, got.index, istar, f"{got.kernel_ms:.1f} ms", flush=True)
    assert got.index == istar and got.energy_i == orc.energy(Q, istar)


def test_arguments(q):
    Q = inputs.uniform_int(20, -9, 9, 2)
    for bad in (dict(k=0), dict(k=13), dict(k=20)):
        with pytest.raises(q.QuboError) as e:
            q.solve_outer(Q, **bad)
        assert e.value.status == -1
    with pytest.raises(q.QuboError) as e:
        q.solve_outer(inputs.normal_fp32(20, 2), 3)
    assert e.value.status == -1
