"""Seeded synthetic QUBO inputs shared by the tests, the smoke check and the benchmark.

This module only draws random numbers and shapes them into instances; it holds
none of the solver's arithmetic.  The paper benchmarks on "a uniformly random
matrix" (Sec. V-C); these generators produce that workload:

* ``uniform_int(n, lo, hi, seed)``: upper-triangular int32 Q including the
  diagonal, entries i.i.d. uniform integers in [lo, hi], lower triangle zero.
* ``normal_fp32(n, seed)``: upper-triangular float32 Q with N(0, 1) entries.
* ``planted(n, lo, hi, seed)``: ``uniform_int`` whose diagonal is rewritten so a
  seeded random x* is the unique ground state (each diagonal entry is
  -(R_i + 1) where x*_i = 1 and +(R_i + 1) where x*_i = 0, with R_i the sum of
  |Q_ij| + |Q_ji| over j != i; any single flip towards x* then lowers the
  energy by at least 1 whatever the other bits are).
* ``edge_int(n, total, seed)``: upper-triangular int32 Q whose absolute entries
  sum to exactly ``total`` (the int32 exactness limit of the solver is
  sum |T| <= 2^30 - 1, so ``total = 2**30 - 1`` sits on it).
* ``batch(count, n_lo, n_hi, seed, kind)``: many instances of uneven size.
* ``poisson_requests(...)``: arrival times and instances for the serving mix.

All draws use ``numpy.random.default_rng(seed)`` (PCG64).
"""
from __future__ import annotations

import numpy as np


def uniform_int(n: int, lo: int, hi: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    Q = rng.integers(lo, hi, size=(n, n), endpoint=True, dtype=np.int64)
    return np.triu(Q).astype(np.int32)


def normal_fp32(n: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    Q = rng.standard_normal(size=(n, n), dtype=np.float64).astype(np.float32)
    return np.triu(Q)


def planted(n: int, lo: int, hi: int, seed: int):
    """Return (Q, xstar) with xstar the unique ground state of Q."""
    rng = np.random.default_rng(seed)
    Q = np.triu(rng.integers(lo, hi, size=(n, n), endpoint=True, dtype=np.int64))
    xstar = rng.integers(0, 2, size=n, dtype=np.int64)
    A = np.abs(Q)
    np.fill_diagonal(A, 0)
    R = A.sum(axis=1) + A.sum(axis=0)
    diag = np.where(xstar == 1, -(R + 1), R + 1)
    np.fill_diagonal(Q, diag)
    if np.abs(Q).max() > 2**31 - 1:
        raise ValueError("planted instance does not fit int32")
    return Q.astype(np.int32), xstar


def edge_int(n: int, total: int, seed: int) -> np.ndarray:
    """Upper-triangular int32 Q (random signs and magnitudes) with sum |Q_ij| == total."""
    rng = np.random.default_rng(seed)
    iu = np.triu_indices(n)
    m = len(iu[0])
    w = rng.random(m) + 0.05
    mag = np.floor(w / w.sum() * total).astype(np.int64)
    short = int(total - mag.sum())              # 0 <= short < m after flooring
    mag[rng.choice(m, size=short, replace=False)] += 1
    sign = np.where(rng.random(m) < 0.5, -1, 1)
    Q = np.zeros((n, n), dtype=np.int64)
    Q[iu] = sign * mag
    assert int(np.abs(Q).sum()) == total and np.abs(Q).max() <= 2**31 - 1
    return Q.astype(np.int32)


def suffix_edge_int(n: int, a: int, total: int, sign: int, seed: int,
                    lo: int = -1000, hi: int = 1000) -> np.ndarray:
    """Upper-triangular int32 Q whose entries in columns j >= a have
    sum |Q_ij| == total, all of sign ``sign`` (+1 or -1; 0: random signs);
    the entries of columns j < a are uniform in [lo, hi]."""
    rng = np.random.default_rng(seed)
    Q = np.triu(rng.integers(lo, hi, size=(n, n), endpoint=True, dtype=np.int64))
    Q[:, a:] = 0
    iu = [(i, j) for j in range(a, n) for i in range(j + 1)]
    w = rng.random(len(iu)) + 0.05
    mag = np.floor(w / w.sum() * total).astype(np.int64)
    mag[rng.choice(len(iu), size=int(total - mag.sum()), replace=False)] += 1
    sg = rng.choice([-1, 1], size=len(iu)) if sign == 0 else np.full(len(iu), sign)
    for (i, j), m, s in zip(iu, mag, sg):
        Q[i, j] = s * m
    assert int(np.abs(Q[:, a:]).sum()) == total
    return Q.astype(np.int32)


def full_int(n: int, lo: int, hi: int, seed: int) -> np.ndarray:
    """Dense int32 Q with BOTH triangles populated (exercises the fold)."""
    rng = np.random.default_rng(seed)
    return rng.integers(lo, hi, size=(n, n), endpoint=True, dtype=np.int64).astype(np.int32)


def batch(count: int, n_lo: int, n_hi: int, seed: int, kind: str = "int",
          lo: int = -100, hi: int = 100):
    """``count`` instances with n ~ U{n_lo..n_hi}; kind 'int' (U[lo,hi]) or 'fp32' (N(0,1))."""
    rng = np.random.default_rng(seed)
    ns = rng.integers(n_lo, n_hi, size=count, endpoint=True)
    seeds = rng.integers(0, 2**62, size=count)
    out = []
    for n, s in zip(ns, seeds):
        if kind == "int":
            out.append(uniform_int(int(n), lo, hi, int(s)))
        elif kind == "fp32":
            out.append(normal_fp32(int(n), int(s)))
        else:
            raise ValueError(kind)
    return out


def poisson_requests(count: int, rate_hz: float, n_lo: int, n_hi: int, seed: int,
                     int_fraction: float = 0.8, lo: int = -100, hi: int = 100):
    """Serving mix: (arrival_s, Q) pairs with Poisson arrivals at ``rate_hz``.

    n ~ U{n_lo..n_hi}; an ``int_fraction`` share is int32 U[lo, hi], the rest
    float32 N(0, 1).
    """
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_hz, size=count)
    arrivals = np.cumsum(gaps) - gaps[0]
    ns = rng.integers(n_lo, n_hi, size=count, endpoint=True)
    is_int = rng.random(size=count) < int_fraction
    seeds = rng.integers(0, 2**62, size=count)
    out = []
    for t, n, ii, s in zip(arrivals, ns, is_int, seeds):
        Q = uniform_int(int(n), lo, hi, int(s)) if ii else normal_fp32(int(n), int(s))
        out.append((float(t), Q))
    return out
