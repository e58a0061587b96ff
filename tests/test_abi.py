"""C ABI and host-side planning, without a GPU.

Checks that the library loads, exports every entry point include/qubo.h
declares, and that the planner (fold, int32 exactness bound, fp32 fixed-point
scale, split and work items) behaves as documented.
"""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2607_04857_amd as q
from paper_2607_04857_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    txt = open(os.path.join(ROOT, "include", "qubo.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(qubo_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    lib = q.lib()
    syms = header_symbols()
    assert len(syms) >= 18
    for s in syms:
        assert hasattr(lib, s), s
    assert sorted(q.EXPORTS) == syms


def test_version_and_last_error():
    assert q.version().startswith("qubo-mi355x")
    assert isinstance(q.lib().qubo_last_error(), bytes)


def test_plan_fold_identity_on_upper_triangular():
    Q = inputs.uniform_int(20, -100, 100, 1)
    info = q.plan_info(Q, tier=2)
    assert np.array_equal(info["T"], Q)
    assert info["sum_abs_t"] == int(np.abs(Q.astype(np.int64)).sum())
    assert info["A"] + info["B"] == 20 and info["B"] == 10
    assert info["items"] == 2 ** (info["A"] - info["L"])


def _suffix_sum(T, A):
    return int(np.abs(T.astype(np.int64)[:, A:]).sum())


def test_packed_tier_eligibility():
    """Tier 4 (two 16-bit chunk energies per word) is planned one suffix bit
    wider than the int32 walk, and only where the sum of |T_ij| over the
    suffix columns bounds every chunk energy within 16 bits."""
    # n = 24, U[-100, 100]: eligible; forced and default plans agree
    Q = inputs.uniform_int(24, -100, 100, 1)
    f = q.plan_info(Q, tier=4)
    assert (f["tier"], f["B"], f["A"]) == (4, 11, 13)
    assert _suffix_sum(f["T"], f["A"]) <= 32767
    d = q.plan_info(Q)
    assert d["tier"] in (1, 2, 4) and d["A"] + d["B"] == 24
    # forced widths: B in [9, 11] for tier 4
    assert q.plan_info(Q, tier=4, B=10)["B"] == 10
    assert q.plan_info(Q, tier=4, B=9, vgpr_levels=12)["B"] == 9
    for bad in (dict(tier=4, B=8), dict(tier=4, B=12), dict(tier=3)):
        with pytest.raises(q.QuboError) as e:
            q.plan_info(Q, **bad)
        assert e.value.status == -1
    # the headline instance's suffix sum is far above the bound: int32 walk
    H = inputs.uniform_int(44, -10000, 10000, 4)
    assert q.plan_info(H)["tier"] == 2
    with pytest.raises(q.QuboError):
        q.plan_info(H, tier=4)
    # float32 input never packs
    F = inputs.normal_fp32(24, 3)
    assert q.plan_info(F)["tier"] != 4
    with pytest.raises(q.QuboError):
        q.plan_info(F, tier=4)
    # too few prefix bits for the wider split
    with pytest.raises(q.QuboError):
        q.plan_info(inputs.uniform_int(16, -100, 100, 2), tier=4)


@pytest.mark.parametrize("sign", [1, -1, 0])
def test_packed_tier_suffix_sum_bound(sign):
    """Suffix-column sum 32767 plans tier 4 whatever the signs (every chunk
    energy lies in [-32767, 32767]); the shift puts the least at -32768."""
    n, B = 22, 11
    Q = inputs.suffix_edge_int(n, n - B, 32767, sign, 30 + sign)
    info = q.plan_info(Q, tier=4)
    assert (info["tier"], info["A"]) == (4, n - B)
    assert _suffix_sum(info["T"], n - B) == 32767
    if sign == 1:                        # all suffix entries positive: least 0
        assert info["pack_shift"] == -32768


def _suffix_diagonal(n, A, d, seed):
    rng = np.random.default_rng(seed)
    Q = np.triu(rng.integers(-1000, 1000, size=(n, n), endpoint=True)).astype(np.int64)
    Q[:, A:] = 0
    for t, v in enumerate(d):
        Q[A + t, A + t] = v
    return Q.astype(np.int32)


@pytest.mark.parametrize("signs", ["pos", "neg", "mixed"])
def test_packed_tier_exact_range_edge(signs):
    """Only the suffix diagonal is set: the chunk energies then span exactly
    the sum of |d_t|.  65535 is the widest range a 16-bit value holds: it
    packs, with the shift that puts the lowest energy at -32768; 65536 does
    not."""
    n, B = 20, 11
    A = n - B
    for total, ok in ((65535, True), (65536, False)):
        d = np.full(B, total // B)
        d[0] += total - d.sum()
        if signs == "neg":
            d = -d
        elif signs == "mixed":
            d[1::2] *= -1
        Q = _suffix_diagonal(n, A, d, 7)
        lo = int(d[d < 0].sum())
        if ok:
            info = q.plan_info(Q, tier=4)
            assert (info["tier"], info["A"]) == (4, A)
            assert info["pack_shift"] == -32768 - lo
            assert q.plan_info(Q)["tier"] == 4
        else:
            with pytest.raises(q.QuboError) as e:
                q.plan_info(Q, tier=4)
            assert e.value.status == -1
            assert q.plan_info(Q)["tier"] != 4


def _chunk_range_brute(T, A):
    """Extremes of E_sd(s, x_p) over every prefix and suffix column, by
    enumeration: E_sd = E(x) - E(x_p alone), from the oracle's own energy
    definition applied to all 2^n states."""
    n = T.shape[0]
    B = n - A
    idx = np.arange(1 << n, dtype=np.int64)
    x = ((idx[:, None] >> (n - 1 - np.arange(n))[None, :]) & 1).astype(np.int64)
    E = np.einsum("si,ij,sj->s", x, T.astype(np.int64), x)
    xp = x.copy()
    xp[:, A:] = 0
    Ep = np.einsum("si,ij,sj->s", xp, T.astype(np.int64), xp)
    esd = E - Ep
    return int(esd.min()), int(esd.max())


@pytest.mark.parametrize("R,seed", [(120, 1), (600, 1), (3000, 1), (3000, 2), (3300, 1),
                                    (5000, 5)])
def test_packed_tier_matches_brute_force_range(R, seed):
    """Tier 4 is planned exactly when the brute-force range of the chunk
    energies (n = 17, all 2^17 states) fits 16 bits, with the shift that
    maps it into [-32768, 32767]."""
    n = 17
    Q = inputs.uniform_int(n, -R, R, 600 + seed)       # ranges 2403 ... 120639
    T = q.plan_info(Q, tier=2)["T"]
    A = n - 11
    lo, hi = _chunk_range_brute(T, A)
    fits = hi - lo <= 65535
    if fits:
        info = q.plan_info(Q, tier=4)
        assert info["A"] == A
        c = info["pack_shift"]
        assert c == -32768 - lo
        assert lo + c == -32768 and hi + c <= 32767
    else:
        with pytest.raises(q.QuboError):
            q.plan_info(Q, tier=4)



def test_plan_fold_moves_lower_triangle_up():
    Q = inputs.full_int(17, -50, 50, 2)
    T = q.plan_info(Q)["T"].astype(np.int64)
    Q64 = Q.astype(np.int64)
    assert np.array_equal(np.tril(T, -1), np.zeros_like(T))
    assert np.array_equal(np.diag(T), np.diag(Q64))
    iu = np.triu_indices(17, 1)
    assert np.array_equal(T[iu], (Q64 + Q64.T)[iu])


def test_int32_exactness_bound():
    n = 16
    lim = 2 ** 30 - 1
    Q = np.zeros((n, n), dtype=np.int32)
    Q[0, 0] = lim                               # sum |T| == 2^30 - 1: accepted
    assert q.plan_info(Q)["sum_abs_t"] == lim
    Q[1, 1] = 1                                 # one more: rejected
    with pytest.raises(q.QuboError) as e:
        q.plan_info(Q)
    assert e.value.status == -2
    # the fold can overflow int32 even when every entry fits: rejected, not wrapped
    Q = np.zeros((n, n), dtype=np.int32)
    Q[0, 1] = Q[1, 0] = 2 ** 31 - 1
    with pytest.raises(q.QuboError):
        q.plan_info(Q)


def test_fp32_fixed_point_scale():
    Q = inputs.normal_fp32(30, 3)
    info = q.plan_info(Q)
    p, T = info["p"], info["T"].astype(np.float64)
    Td = np.triu(Q.astype(np.float64)) + np.tril(Q.astype(np.float64), -1).T
    S = np.abs(Td).sum()
    assert S * 2.0 ** p <= 2 ** 29 < S * 2.0 ** (p + 1)
    assert np.all(np.abs(T - Td * 2.0 ** p) <= 0.5)
    nnz = int(np.count_nonzero(Td))
    assert info["eps_q"] == pytest.approx(nnz * 2.0 ** (-p - 1))
    assert info["sum_abs_t"] <= 2 ** 29 + nnz / 2
    assert info["eps_q"] * 2 <= 1e-5 * np.abs(Q.astype(np.float64)).sum()


@pytest.mark.parametrize("S,p", [(2.0 ** 20, 9), (2.0 ** 20 + 1, 8), (2.0 ** 20 - 1, 9),
                                 (0.75, 29), (0.5, 30), (2.0 ** 29, 0), (2.0 ** 29 + 64, -1)])
def test_fp32_exponent_at_powers_of_two(S, p):
    """p is the largest exponent with S 2^p <= 2^29 exactly, also where
    2^29 / S is a power of two or one unit of rounding away from one (a
    single float32 entry on the diagonal: S = |Q_00|)."""
    Q = np.zeros((3, 3), dtype=np.float32)
    Q[0, 0] = np.float32(-S)
    assert float(Q[0, 0]) == -S
    info = q.plan_info(Q)
    assert info["p"] == p
    assert S * 2.0 ** p <= 2 ** 29 < S * 2.0 ** (p + 1)


@pytest.mark.parametrize("n,full", [(60, False), (60, True), (46, False), (20, True)])
def test_fp32_tolerance_bound(n, full):
    """tol = 2 eps_q = nnz 2^-p, and p is the largest exponent with
    S 2^p <= 2^29 (S = sum |T|), so tol < nnz S / 2^28 <= n(n+1)/2 * sum|Q| / 2^28:
    at most 6.9e-6 sum|Q| for every n <= 60, under the 1e-5 bound."""
    rng = np.random.default_rng(n)
    Q = rng.standard_normal((n, n)).astype(np.float32)
    if not full:
        Q = np.triu(Q)
    info = q.plan_info(Q)
    T = np.triu(Q.astype(np.float64)) + np.tril(Q.astype(np.float64), -1).T
    S = np.abs(T).sum()
    nnz = int(np.count_nonzero(T))
    tol = 2 * info["eps_q"]
    assert tol == pytest.approx(nnz * 2.0 ** -info["p"])
    assert tol < nnz * S / 2 ** 28
    sq = float(np.abs(Q.astype(np.float64)).sum())
    assert tol < n * (n + 1) / 2 * sq / 2 ** 28 <= 6.9e-6 * sq


def test_fp32_zero_and_nonfinite():
    assert q.plan_info(np.zeros((16, 16), dtype=np.float32))["p"] == 0
    Q = inputs.normal_fp32(16, 4)
    Q[3, 5] = np.nan
    with pytest.raises(q.QuboError) as e:
        q.plan_info(Q)
    assert e.value.status == -3
    Q[3, 5] = np.inf
    with pytest.raises(q.QuboError):
        q.plan_info(Q)


@pytest.mark.parametrize("n", [1, 7, 14])
def test_tiny_instances_take_the_direct_path(n):
    info = q.plan_info(inputs.uniform_int(n, -9, 9, n))
    assert info["direct"] == 1 and info["items"] == 0


def test_split_options_and_validation():
    Q = inputs.uniform_int(24, -100, 100, 5)
    for B in (6, 8, 10):
        info = q.plan_info(Q, B=B, L=7)
        assert (info["B"], info["A"], info["L"]) == (B, 24 - B, 7)
        assert info["items"] == 2 ** (24 - B - 7)
    for bad in (dict(B=5), dict(B=11), dict(L=5), dict(L=30), dict(tier=3)):
        with pytest.raises(q.QuboError) as e:
            q.plan_info(Q, **bad)
        assert e.value.status == -1


def test_bad_n():
    for n in (0, 61):
        with pytest.raises((q.QuboError, ValueError)):
            q.plan_info(np.zeros((max(n, 1), max(n, 1)), dtype=np.int32)[:n, :n])


def test_headline_plan_is_provably_exact():
    info = q.plan_info(inputs.uniform_int(44, -10000, 10000, 4))
    assert info["sum_abs_t"] <= 990 * 10000 < 2 ** 30 - 1
    assert (info["A"], info["B"]) == (34, 10)


@pytest.mark.skipif(os.environ.get("HIP_VISIBLE_DEVICES") is None and
                    __import__("torch").cuda.is_available(), reason="GPU present")
def test_solve_without_gpu_fails_loudly():
    with pytest.raises(q.QuboError) as e:
        q.solve(inputs.uniform_int(16, -5, 5, 1))
    assert e.value.status == -5


def test_topk_argument_checks_need_no_gpu():
    import paper_2607_04857_amd as q
    Q = np.zeros((3, 3), dtype=np.int32)
    for k in (9, 1025, -1):
        with pytest.raises(q.QuboError) as ei:
            q.solve(Q, k=k)
        assert ei.value.status == -1


def test_item_range_options_validated_on_host():
    import paper_2607_04857_amd as q
    Q = inputs.uniform_int(24, -100, 100, 5)
    info = q.plan_info(Q)
    ok = q.plan_info(Q, item_first=info["items"] - 2, item_count=2)
    assert ok["items"] == info["items"]
    for first, count in [(info["items"] - 1, 2), (-1, 1), (0, -3), (3, 0)]:
        with pytest.raises(q.QuboError) as ei:
            q.plan_info(Q, item_first=first, item_count=count)
        assert ei.value.status == -1
    with pytest.raises(q.QuboError):
        q.plan_info(inputs.uniform_int(12, -100, 100, 5), item_first=0, item_count=1)


def test_header_is_plain_c(tmp_path):
    """include/qubo.h is a C ABI: it compiles as C99 with warnings as errors."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "use_header.c"
    src.write_text('#include "qubo.h"\n'
                   "int main(void) { qubo_result_t r; qubo_checkpoint_t c; qubo_tune_entry_t e;\n"
                   "  (void)r; (void)c; (void)e; return (int)sizeof(qubo_options_t) == 32 ? 0 : 1; }\n")
    subprocess.run([cc, "-std=c99", "-Wall", "-Wextra", "-Werror", "-fsyntax-only",
                    "-I", os.path.join(ROOT, "include"), str(src)], check=True)


@pytest.mark.parametrize("n,k,seed", [(9, 3, 1), (11, 1, 2), (12, 5, 3)])
def test_outer_reduction_identity(orc, n, k, seed):
    """E(x_f, x_r) = c(x_f) + E_Qr(x_r) for every outer assignment and every
    x_r, by the oracle's direct energy of both sides (full matrix input, so
    the fold is exercised); and on upper-triangular input Qr is the paper's
    Q_rr + diag(x_f Q_fr)."""
    rng = np.random.default_rng(seed)
    Q = rng.integers(-50, 51, (n, n)).astype(np.int32)
    m = n - k
    for xf in range(1 << k):
        Qr, c = q.reduce_outer(Q, k, xf)
        assert np.all(np.tril(Qr, -1) == 0)
        for xr in range(1 << m):
            assert orc.energy(Q, (xf << m) | xr) == c + orc.energy(Qr, xr)
    U = np.triu(Q)
    for xf in (0, (1 << k) - 1, 1 % (1 << k)):
        x_f = np.array([(xf >> (k - 1 - i)) & 1 for i in range(k)], dtype=np.int64)
        Qr, c = q.reduce_outer(U, k, xf)
        want = U[k:, k:].astype(np.int64) + np.diag(x_f @ U[:k, k:].astype(np.int64))
        assert np.array_equal(Qr, want)
        assert c == int(x_f @ U[:k, :k].astype(np.int64) @ x_f)


def test_outer_reduction_arguments():
    Q = inputs.uniform_int(10, -9, 9, 1)
    for bad in (dict(k=0, xf=0), dict(k=10, xf=0), dict(k=3, xf=8)):
        with pytest.raises(q.QuboError) as e:
            q.reduce_outer(Q, **bad)
        assert e.value.status == -1
    big = np.zeros((4, 4), dtype=np.int32)
    big[0, 3] = 2 ** 31 - 1
    big[1, 3] = 2 ** 31 - 1        # x_0 = x_1 = 1 puts 2^32 - 2 on Qr's diagonal
    with pytest.raises(q.QuboError) as e:
        q.reduce_outer(big, 2, 3)
    assert e.value.status == -2
    with pytest.raises(TypeError):
        q.reduce_outer(Q.astype(np.float32), 2, 0)


@pytest.mark.parametrize("kind,seed", [("int", 1), ("int", 2), ("fp32", 3)])
def test_int32_walk_shift_is_least_chunk_energy(kind, seed):
    """The int32 walk adds c = -(least chunk energy of its split) to every
    chunk energy, so they start at 0; c from the brute-force range over all
    2^17 states (the float32 case on its fixed-point image)."""
    n = 17
    Q = inputs.uniform_int(n, -5000, 5000, 640 + seed) if kind == "int" \
        else inputs.normal_fp32(n, 640 + seed)
    info = q.plan_info(Q, tier=2)
    assert info["tier"] == 2
    lo, hi = _chunk_range_brute(info["T"], info["A"])
    assert info["pack_shift"] == -lo
    assert info["sum_abs_t"] + abs(lo) <= 2 ** 30 - 1


def test_int32_walk_shift_respects_the_exactness_bound():
    """At sum |T| = 2^30 - 1 no shift fits the int32 bound: c = 0.  Well
    inside it, c = -(least chunk energy), within the bound."""
    n = 17
    edge = q.plan_info(inputs.edge_int(n, 2 ** 30 - 1, 5), tier=2)
    assert edge["sum_abs_t"] == 2 ** 30 - 1 and edge["pack_shift"] == 0
    half = q.plan_info(inputs.edge_int(n, 2 ** 28, 5), tier=2)
    lo, _ = _chunk_range_brute(half["T"], half["A"])
    assert lo < 0 and half["pack_shift"] == -lo
    assert half["sum_abs_t"] - lo <= 2 ** 30 - 1
