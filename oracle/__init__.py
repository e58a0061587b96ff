"""CPU oracle for exhaustive dense-QUBO minimisation (test infrastructure).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU solver never calls it, and it
shares no code with the GPU solver: it is the plain definition that GPU
results are checked against.

What it computes (see ``qubo_oracle.c`` for the C side):

* ``energy(Q, index)``  -- E(x) = sum_{i,j} Q_ij x_i x_j (the QUBO objective of
  the paper's Introduction) for the state ``x`` that is row ``index`` of the
  lexicographic state matrix U_N (Sec. II-B: column 0 is the most significant
  bit, so x_i = (index >> (n-1-i)) & 1).
* ``solve(Q, k)`` (O1) -- direct evaluation of every state (the naive
  brute force of Sec. I-D); returns the k lexicographically smallest
  (E, index) pairs, i.e. the minimum energy with its lowest index first.
* ``solve_range(Q, first, count, k)`` -- the same over an index range.
* ``gray_solve(Q)`` (O2) -- the textbook O(N 2^N) Gray-code brute force with
  local fields (Sec. I-D), best pair only.
* ``gray_solve_range(Q, i0, i1)`` -- the same walk over the Gray indices
  [i0, i1), i.e. the states i ^ (i >> 1), so that a long walk can be split
  into shards and resumed.

int32 input is summed exactly in int64; fp32 input is converted exactly to
float64 and summed in float64.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "qubo_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libqubo_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into ``oracle/libqubo_oracle.so``."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(
            ["gcc", "-O3", "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC", "-pthread",
             _SRC, "-o", tmp])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build(force=False)
    lib = ctypes.CDLL(_LIB_PATH)
    c_i32p = ctypes.POINTER(ctypes.c_int32)
    c_f32p = ctypes.POINTER(ctypes.c_float)
    c_i64p = ctypes.POINTER(ctypes.c_int64)
    c_f64p = ctypes.POINTER(ctypes.c_double)
    c_u64p = ctypes.POINTER(ctypes.c_uint64)
    u64, i32 = ctypes.c_uint64, ctypes.c_int
    lib.oracle_energy_i.argtypes = [i32, c_i32p, u64, c_i64p]
    lib.oracle_energy_f.argtypes = [i32, c_f32p, u64, c_f64p]
    lib.oracle_solve_i.argtypes = [i32, c_i32p, u64, u64, i32, i32, c_i64p, c_u64p]
    lib.oracle_solve_f.argtypes = [i32, c_f32p, u64, u64, i32, i32, c_f64p, c_u64p]
    lib.oracle_gray_i.argtypes = [i32, c_i32p, i32, c_i64p, c_u64p]
    lib.oracle_gray_f.argtypes = [i32, c_f32p, i32, c_f64p, c_u64p]
    lib.oracle_gray_range_i.argtypes = [i32, c_i32p, u64, u64, i32, c_i64p, c_u64p]
    lib.oracle_gray_range_f.argtypes = [i32, c_f32p, u64, u64, i32, c_f64p, c_u64p]
    for f in (lib.oracle_energy_i, lib.oracle_energy_f, lib.oracle_solve_i,
              lib.oracle_solve_f, lib.oracle_gray_i, lib.oracle_gray_f,
              lib.oracle_gray_range_i, lib.oracle_gray_range_f):
        f.restype = ctypes.c_int
    lib.oracle_default_threads.argtypes = []
    lib.oracle_default_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _prep(Q):
    Q = np.asarray(Q)
    if Q.ndim != 2 or Q.shape[0] != Q.shape[1]:
        raise ValueError("Q must be a square matrix")
    if Q.dtype == np.float32:
        return np.ascontiguousarray(Q), False
    if Q.dtype.kind in "iu":
        if Q.size and (Q.min() < -2**31 or Q.max() > 2**31 - 1):
            raise ValueError("integer Q must fit int32")
        return np.ascontiguousarray(Q, dtype=np.int32), True
    raise TypeError("Q must be int32 or float32")


def _ptr(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def default_threads() -> int:
    return _load().oracle_default_threads()


def energy(Q, index: int):
    """E(x) of the state with U_N row ``index`` (int for int Q, float for fp32)."""
    lib = _load()
    Qc, is_int = _prep(Q)
    n = Qc.shape[0]
    if is_int:
        out = ctypes.c_int64()
        rc = lib.oracle_energy_i(n, _ptr(Qc, ctypes.c_int32), int(index), ctypes.byref(out))
    else:
        out = ctypes.c_double()
        rc = lib.oracle_energy_f(n, _ptr(Qc, ctypes.c_float), int(index), ctypes.byref(out))
    if rc != 0:
        raise ValueError("oracle_energy failed")
    return int(out.value) if is_int else float(out.value)


def solve_range(Q, first: int, count: int, k: int = 1, threads: int = 0):
    """k smallest (E, index) pairs over indices [first, first+count) (O1)."""
    lib = _load()
    Qc, is_int = _prep(Q)
    n = Qc.shape[0]
    idx = np.zeros(k, dtype=np.uint64)
    if is_int:
        E = np.zeros(k, dtype=np.int64)
        rc = lib.oracle_solve_i(n, _ptr(Qc, ctypes.c_int32), int(first), int(count), int(k),
                                int(threads), _ptr(E, ctypes.c_int64), _ptr(idx, ctypes.c_uint64))
    else:
        E = np.zeros(k, dtype=np.float64)
        rc = lib.oracle_solve_f(n, _ptr(Qc, ctypes.c_float), int(first), int(count), int(k),
                                int(threads), _ptr(E, ctypes.c_double), _ptr(idx, ctypes.c_uint64))
    if rc != 0:
        raise ValueError(f"oracle_solve failed ({rc})")
    m = min(k, int(count))
    pairs = [(int(E[q]) if is_int else float(E[q]), int(idx[q])) for q in range(m)]
    return pairs


def solve(Q, k: int = 1, threads: int = 0):
    """k smallest (E, index) pairs over all 2^n states (O1)."""
    n = np.asarray(Q).shape[0]
    return solve_range(Q, 0, 1 << n, k, threads)


def gray_solve(Q, threads: int = 0):
    """Best (E, index) pair over all 2^n states by the local-field Gray walk (O2)."""
    lib = _load()
    Qc, is_int = _prep(Q)
    n = Qc.shape[0]
    idx = ctypes.c_uint64()
    if is_int:
        E = ctypes.c_int64()
        rc = lib.oracle_gray_i(n, _ptr(Qc, ctypes.c_int32), int(threads), ctypes.byref(E),
                               ctypes.byref(idx))
    else:
        E = ctypes.c_double()
        rc = lib.oracle_gray_f(n, _ptr(Qc, ctypes.c_float), int(threads), ctypes.byref(E),
                               ctypes.byref(idx))
    if rc != 0:
        raise ValueError(f"oracle_gray failed ({rc})")
    return (int(E.value) if is_int else float(E.value), int(idx.value))


def gray_solve_range(Q, i0: int, i1: int, threads: int = 0):
    """Best (E, index) pair over the states of Gray indices [i0, i1) (O2 shard)."""
    lib = _load()
    Qc, is_int = _prep(Q)
    n = Qc.shape[0]
    idx = ctypes.c_uint64()
    if is_int:
        E = ctypes.c_int64()
        rc = lib.oracle_gray_range_i(n, _ptr(Qc, ctypes.c_int32), int(i0), int(i1), int(threads),
                                     ctypes.byref(E), ctypes.byref(idx))
    else:
        E = ctypes.c_double()
        rc = lib.oracle_gray_range_f(n, _ptr(Qc, ctypes.c_float), int(i0), int(i1), int(threads),
                                     ctypes.byref(E), ctypes.byref(idx))
    if rc != 0:
        raise ValueError(f"oracle_gray_range failed ({rc})")
    return (int(E.value) if is_int else float(E.value), int(idx.value))


def state_of(index: int, n: int) -> np.ndarray:
    """x as a 0/1 vector for U_N row ``index`` (x_0 is the most significant bit)."""
    return np.array([(int(index) >> (n - 1 - i)) & 1 for i in range(n)], dtype=np.int64)


def index_of(x) -> int:
    """U_N row of the 0/1 vector ``x`` (x_0 is the most significant bit)."""
    r = 0
    for b in x:
        r = (r << 1) | int(b)
    return r
