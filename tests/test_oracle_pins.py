"""Pins of the CPU oracle against values fixed by the paper and by mathematics.

None of these tests compares the oracle with itself: each checks it against a
hand-derived table, a closed form, a construction with a proven answer, an
independent formulation (the matrix form of Sec. II-A evaluated with numpy),
or an invariance of the objective.
"""
import itertools

import numpy as np
import pytest

from conftest import read_table
from paper_2607_04857_amd import inputs


def _golden_Q(header):
    n = int(header["n"][0])
    return np.array([int(v) for v in header["Q"]], dtype=np.int32).reshape(n, n)


@pytest.mark.parametrize("name", ["p8_worked_example.txt", "fold_full_matrix.txt",
                                  "tie_lowest_index.txt"])
def test_hand_tables(orc, name):
    header, rows = read_table(name)
    Q = _golden_Q(header)
    n = Q.shape[0]
    table = {int(r[0]): int(r[2]) for r in rows}
    for idx, E in table.items():
        x = rows[idx][1]
        assert int(x, 2) == idx                     # index is the MSB-left binary row
        assert orc.energy(Q, idx) == E
    expect = sorted((E, idx) for idx, E in table.items())
    for threads in (1, 3):
        assert orc.solve(Q, k=len(expect), threads=threads) == expect
    assert orc.gray_solve(Q, threads=1) == expect[0]
    assert orc.gray_solve(Q, threads=2) == expect[0]
    if "best" in header:
        assert expect[0] == (int(header["best"][0]), int(header["best"][1]))
    assert len(table) == 2 ** n


def test_fold_transpose_invariance(orc):
    """E over all i, j is unchanged by moving entries across the diagonal."""
    Q = inputs.full_int(9, -50, 50, seed=11)
    U = np.triu(Q) + np.tril(Q, -1).T           # fold lower into upper
    L = np.tril(Q) + np.triu(Q, 1).T            # fold upper into lower
    for idx in range(0, 512, 7):
        e = orc.energy(Q, idx)
        assert e == orc.energy(U, idx) == orc.energy(L, idx) == orc.energy(Q.T.copy(), idx)
    assert orc.solve(Q, k=5) == orc.solve(U, k=5) == orc.solve(L, k=5)


def test_matrix_form_all_states(orc):
    """Oracle energies equal diag(X Q X^T) (Sec. II-A, Eq. total_energy) for every state."""
    for n, seed in [(1, 1), (2, 2), (5, 3), (8, 4), (10, 5)]:
        Q = inputs.full_int(n, -1000, 1000, seed)
        X = np.array(list(itertools.product([0, 1], repeat=n)), dtype=np.int64)  # U_N rows
        E = np.einsum("mi,ij,mj->m", X, Q.astype(np.int64), X)
        got = np.array([orc.energy(Q, r) for r in range(2 ** n)])
        assert np.array_equal(got, E)
        order = np.lexsort((np.arange(2 ** n), E))
        assert orc.solve(Q, k=1) == [(int(E[order[0]]), int(order[0]))]


def test_matrix_form_fp32(orc):
    Q = inputs.normal_fp32(9, seed=7)
    X = np.array(list(itertools.product([0, 1], repeat=9)), dtype=np.float64)
    E = np.einsum("mi,ij,mj->m", X, Q.astype(np.float64), X)
    got = np.array([orc.energy(Q, r) for r in range(512)])
    assert np.allclose(got, E, rtol=0, atol=1e-12 * np.abs(Q).sum())
    best = orc.solve(Q, k=1)[0]
    assert best[1] == int(np.argmin(E))
    assert orc.gray_solve(Q)[1] == best[1]


@pytest.mark.parametrize("n,seed", [(1, 0), (6, 1), (13, 2), (17, 3)])
def test_p1_diagonal_closed_form(orc, n, seed):
    """Diagonal-only Q: E* = sum_i min(0, Q_ii); the lowest-index argmin sets x_i iff Q_ii < 0."""
    rng = np.random.default_rng(seed)
    d = rng.integers(-5, 5, size=n, endpoint=True)
    d[rng.random(n) < 0.3] = 0                      # zero diagonals must stay 0 in the argmin
    Q = np.diag(d).astype(np.int32)
    Estar = int(np.minimum(d, 0).sum())
    xstar = (d < 0).astype(int)
    idx = int("".join(map(str, xstar)), 2)
    assert orc.solve(Q, k=1, threads=3) == [(Estar, idx)]
    assert orc.gray_solve(Q, threads=3) == (Estar, idx)
    Qf = Q.astype(np.float32) * np.float32(0.25)
    assert orc.solve(Qf, k=1) == [(Estar * 0.25, idx)]


@pytest.mark.parametrize("n,seed", [(5, 1), (12, 2), (16, 3)])
def test_p2_planted_unique(orc, n, seed):
    """Planted instance: x* is the unique minimum and E(x) >= E(x*) + Hamming(x, x*)."""
    Q, xstar = inputs.planted(n, -100, 100, seed)
    istar = int("".join(map(str, xstar)), 2)
    top = orc.solve(Q, k=2, threads=2)
    assert top[0][1] == istar
    assert top[1][0] >= top[0][0] + 1
    assert orc.gray_solve(Q) == top[0]
    if n <= 12:
        for r in range(2 ** n):
            ham = bin(r ^ istar).count("1")
            assert orc.energy(Q, r) >= top[0][0] + ham


def test_p3_single_flip_identity(orc):
    """E(x ^ e_k) - E(x) = (1 - 2 x_k) (Q_kk + sum_{j != k} (Q_kj + Q_jk) x_j)."""
    n = 11
    Q = inputs.full_int(n, -300, 300, seed=5).astype(np.int64)
    rng = np.random.default_rng(0)
    for r in rng.integers(0, 2 ** n, size=40):
        x = orc.state_of(int(r), n)
        for k in range(n):
            f = Q[k, k] + sum((Q[k, j] + Q[j, k]) * x[j] for j in range(n) if j != k)
            flipped = int(r) ^ (1 << (n - 1 - k))
            assert orc.energy(Q, flipped) - orc.energy(Q, int(r)) == (1 - 2 * x[k]) * f


@pytest.mark.parametrize("n,seed", [(3, 1), (14, 2), (20, 3)])
def test_o1_equals_o2_int(orc, n, seed):
    Q = inputs.full_int(n, -1000, 1000, seed)
    assert orc.solve(Q, k=1) == [orc.gray_solve(Q)]


@pytest.mark.parametrize("n,seed", [(10, 1), (18, 2)])
def test_o1_vs_o2_fp32(orc, n, seed):
    Q = inputs.normal_fp32(n, seed)
    e1, i1 = orc.solve(Q, k=1)[0]
    e2, i2 = orc.gray_solve(Q)
    assert i1 == i2
    assert abs(e1 - e2) <= 1e-9 * np.abs(Q.astype(np.float64)).sum()


def test_p6_permutation(orc):
    """Relabelling variables permutes the argmin and keeps E* (Sec. II-D)."""
    n = 14
    Q = inputs.uniform_int(n, -100, 100, seed=21)
    E, idx = orc.solve(Q, k=1)[0]
    x = orc.state_of(idx, n)
    perm = np.random.default_rng(3).permutation(n)
    Qp = Q[np.ix_(perm, perm)].copy()                # variable i of Qp is variable perm[i] of Q
    Ep, idxp = orc.solve(Qp, k=1)[0]
    assert Ep == E
    xp = orc.state_of(idxp, n)
    assert orc.energy(Q, orc.index_of(xp[np.argsort(perm)])) == E
    assert orc.energy(Qp, orc.index_of(x[perm])) == E


def test_p6_negation_and_scaling(orc):
    n = 12
    Q = inputs.uniform_int(n, -100, 100, seed=22)
    E, idx = orc.solve(Q, k=1)[0]
    for c in (2, 7):
        assert orc.solve(Q * c, k=1) == [(c * E, idx)]
    neg = orc.solve(-Q, k=1)[0]                       # min E(-Q) = -max E(Q)
    allE = [orc.energy(Q, r) for r in range(2 ** n)]
    assert neg[0] == -max(allE)
    assert neg[1] == allE.index(max(allE))


def test_q_prime_reduction(orc):
    """Sec. III-C.1: fixing the first k bits gives Q' = Q_rr + diag(x_f Q_fr) and c(x_f)."""
    n, kf = 12, 3
    Q = inputs.uniform_int(n, -100, 100, seed=23).astype(np.int64)
    best = orc.solve(Q.astype(np.int32), k=1)[0]
    cands = []
    for f in range(2 ** kf):
        xf = orc.state_of(f, kf)
        Qrr = Q[kf:, kf:].copy()
        Qrr[np.diag_indices(n - kf)] += xf @ Q[:kf, kf:]
        c = int(xf @ Q[:kf, :kf] @ xf)
        e, r = orc.solve(Qrr.astype(np.int32), k=1)[0]
        cands.append((c + e, (f << (n - kf)) | r))
    assert min(cands) == best


def test_range_and_topk(orc):
    header, rows = read_table("p8_worked_example.txt")
    Q = _golden_Q(header)
    table = {int(r[0]): int(r[2]) for r in rows}
    for first, count in [(0, 16), (4, 4), (8, 8), (13, 1), (5, 10)]:
        expect = sorted((table[i], i) for i in range(first, first + count))
        assert orc.solve_range(Q, first, count, k=count, threads=2) == expect
    assert orc.solve_range(Q, 0, 16, k=20)[:16] == sorted((E, i) for i, E in table.items())


def test_zero_and_degenerate(orc):
    Z = np.zeros((9, 9), dtype=np.int32)
    assert orc.solve(Z, k=3) == [(0, 0), (0, 1), (0, 2)]
    assert orc.gray_solve(Z) == (0, 0)
    assert orc.solve(np.array([[5]], dtype=np.int32)) == [(0, 0)]
    assert orc.solve(np.array([[-5]], dtype=np.int32)) == [(-5, 1)]
    neg = np.full((6, 6), -1, dtype=np.int32)
    assert orc.solve(neg) == [(-36, 63)]


def test_gray3_paper_figure(orc):
    """Sec. III-B, Fig. "3-bit Gray code sequence": step i visits g(i) = i ^ (i >> 1), and
    step i -> i + 1 flips vector position k = 3 - 1 - ctz(i + 1) (MSB-left).  O2's
    Gray-index range entry walks exactly the states the figure lists for that range."""
    _, rows = read_table("gray3.txt")
    codes = [r[1] for r in rows]
    assert [int(r[0]) for r in rows] == list(range(8))
    for i, code in enumerate(codes):
        assert code == format(i ^ (i >> 1), "03b")
        if i + 1 < 8:
            diff = [p for p in range(3) if code[p] != codes[i + 1][p]]
            ctz = ((i + 1) & -(i + 1)).bit_length() - 1
            assert diff == [3 - 1 - ctz]
    Q = np.diag([-4, -2, -1]).astype(np.int32)       # E(x) = -index, so the minimum names the
    for i0 in range(8):                              # largest row the walk visited
        for i1 in range(i0 + 1, 9):
            top = max(int(c, 2) for c in codes[i0:i1])
            for threads in (1, 2):
                assert orc.gray_solve_range(Q, i0, i1, threads=threads) == (-top, top)


@pytest.mark.parametrize("threads", [1, 3])
def test_gray_range_equals_direct(orc, threads):
    """O2 over a Gray-index range [i0, i1) = the direct minimum over the states g(i) in it."""
    n = 12
    Q = inputs.full_int(n, -500, 500, seed=31)
    Qf = inputs.normal_fp32(n, seed=32)
    rng = np.random.default_rng(5)
    ranges = [(0, 1), (0, 2 ** n), (2 ** n - 1, 2 ** n), (1000, 1001)]
    ranges += [tuple(sorted(rng.choice(2 ** n + 1, size=2, replace=False))) for _ in range(6)]
    for i0, i1 in ranges:
        states = [i ^ (i >> 1) for i in range(i0, i1)]
        exp = min((orc.energy(Q, g), g) for g in states)
        assert orc.gray_solve_range(Q, i0, i1, threads=threads) == exp
        ef, gf = min((orc.energy(Qf, g), g) for g in states)
        got = orc.gray_solve_range(Qf, i0, i1, threads=threads)
        assert got[1] == gf and abs(got[0] - ef) <= 1e-9 * np.abs(Qf.astype(np.float64)).sum()
