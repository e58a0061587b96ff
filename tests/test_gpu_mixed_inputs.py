"""GPU parity on a seeded spread of input shapes: value ranges from +-1
(thousands of tied states) to the int32 exactness edge, mostly-zero and
all-zero matrices, every split B the planner allows and both walk tiers,
checked state by state against the oracle (int32 exactly, float32 by its
own rescoring)."""
import numpy as np
import pytest

from conftest import check_fp32
from paper_2607_04857_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def q():
    import paper_2607_04857_amd as q
    q.lib()
    return q


def _case(kind, n, seed):
    rng = np.random.default_rng(seed)
    if kind == "pm1":
        return np.triu(rng.integers(-1, 2, (n, n))).astype(np.int32)
    if kind == "sparse":
        Q = np.triu(rng.integers(-1000, 1001, (n, n)))
        return (Q * (rng.random((n, n)) < 0.1)).astype(np.int32)
    if kind == "zero":
        return np.zeros((n, n), dtype=np.int32)
    if kind == "edge":
        return inputs.edge_int(n, (1 << 30) - 1, seed)
    if kind == "negdiag":     # every single variable wants to be 1, couplings push back
        Q = np.triu(rng.integers(0, 50, (n, n)))
        np.fill_diagonal(Q, -rng.integers(100, 400, n))
        return Q.astype(np.int32)
    if kind == "full":        # both triangles set: the fold matters
        return rng.integers(-3000, 3001, (n, n)).astype(np.int32)
    raise ValueError(kind)


CASES = [(kind, n, 100 * i + n) for i, kind in enumerate(
    ("pm1", "sparse", "zero", "edge", "negdiag", "full")) for n in (15, 18, 21)]


@pytest.mark.parametrize("kind,n,seed", CASES)
@pytest.mark.parametrize("tier", [1, 2])
def test_int32_cases(q, orc, kind, n, seed, tier):
    Q = _case(kind, n, seed)
    exp = orc.solve(Q, k=1)[0]
    for B in (6, 8, 10):
        if n - B < 6:
            continue
        got = q.solve(Q, B=B, tier=tier)
        assert (got.energy_i, got.index) == exp, (kind, n, B, tier, got, exp)


@pytest.mark.parametrize("n,seed", [(16, 1), (19, 2), (22, 3)])
def test_fp32_cases(q, orc, n, seed):
    Q = inputs.normal_fp32(n, 500 + seed)
    Q[np.abs(Q) < 0.5] = 0.0                      # many exact zeros
    E, idx = orc.solve(Q, k=1)[0]
    for tier in (1, 2):
        check_fp32(orc, Q, q.solve(Q, tier=tier), E, idx)
