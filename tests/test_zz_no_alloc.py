"""The allocation-free entry point (qubo_solve_noalloc) against qubo_solve.

Both run the same plan and kernels; the allocation-free call keeps the job
in the library's per-device scratch array.  Results must be identical to
qubo_solve's (int32: exact energy and lowest index; float32: the same
integer solve and float64 rescore) and to the oracle, on consecutive calls
whose inputs shrink (the scratch keeps the previous call's contents, which
must not leak into the next result), and a plan too large for the scratch
is refused before any device work.
"""
import ctypes

import numpy as np
import pytest

from conftest import check_fp32
from paper_2607_04857_amd import inputs

pytestmark = pytest.mark.gpu


def _same(a, b):
    return (a.energy_i, a.index, a.p, a.A, a.B, a.L, a.tier) == \
        (b.energy_i, b.index, b.p, b.A, b.B, b.L, b.tier) and a.energy == b.energy


def test_noalloc_matches_solve_on_shrinking_inputs(orc):
    import paper_2607_04857_amd as q
    assert q.noalloc_scratch_bytes() == 16 << 20
    cases = [inputs.uniform_int(36, -1000, 1000, 2),          # walk, 2^36 states
             inputs.uniform_int(24, -100, 100, 1),            # smaller walk
             inputs.normal_fp32(26, 8),                       # float32, smaller again
             inputs.uniform_int(12, -100, 100, 5),            # direct evaluation
             np.zeros((18, 18), dtype=np.int32)]              # ties: index 0
    for k, Q in enumerate(cases):
        n = Q.shape[0]
        print(f"noalloc call {k}: n={n} {Q.dtype}", flush=True)
        got = q.solve_noalloc(Q)
        ref = q.solve(Q)
        assert _same(got, ref), (k, got, ref)
        if n <= 26:
            E, idx = orc.solve(Q, k=1)[0]
            if Q.dtype == np.int32:
                assert (got.energy_i, got.index) == (E, idx)
            else:
                check_fp32(orc, Q, got, E, idx)


def test_noalloc_on_a_caller_stream_twice():
    """On a stream of the caller's (made with the HIP runtime the library is
    linked against, so no second runtime enters the process)."""
    import paper_2607_04857_amd as q
    q.lib()
    hip = ctypes.CDLL("libamdhip64.so.7")
    s = ctypes.c_void_p()
    assert hip.hipStreamCreateWithFlags(ctypes.byref(s), ctypes.c_uint(1)) == 0   # non-blocking
    try:
        big = inputs.uniform_int(40, -10000, 10000, 3)
        small = inputs.uniform_int(30, -1000, 1000, 10)
        for Q in (big, small):
            print(f"noalloc on a caller stream: n={Q.shape[0]}", flush=True)
            out = q._Result()
            assert q.lib().qubo_solve_noalloc(Q.ctypes.data, Q.shape[0], 0, s,
                                              ctypes.byref(out)) == 0
            got = q._result(out, Q.shape[0])
            assert _same(got, q.solve(Q))
    finally:
        hip.hipStreamDestroy(s)


def test_noalloc_rejects_plans_beyond_the_scratch():
    """Default plans hold at most 2^18 work items (4 MiB of item records) for
    every n <= 60 and fit; a tuned plan with 2^20 items at n = 56 does not."""
    import paper_2607_04857_amd as q
    Q = inputs.uniform_int(56, -100, 100, 56)
    assert q.plan_info(Q)["items"] == 1 << 18
    q.tune_set([{"n": 56, "dtype": "int32", "B": 10, "L": 26, "tier": 2, "vgpr_levels": 4}])
    try:
        info = q.plan_info(Q)
        assert info["items"] == 1 << 20
        assert info["items"] * 16 >= q.noalloc_scratch_bytes()    # item records alone fill it
        with pytest.raises(q.QuboError) as e:
            q.solve_noalloc(Q)
        assert e.value.status == -4 and "scratch" in e.value.message
    finally:
        q.tune_clear()
    # the refusal left the scratch usable
    Q2 = inputs.uniform_int(22, -100, 100, 22)
    assert _same(q.solve_noalloc(Q2), q.solve(Q2))


def test_noalloc_argument_errors():
    import paper_2607_04857_amd as q
    out = q._Result()
    lib = q.lib()
    assert lib.qubo_solve_noalloc(None, 10, 0, None, ctypes.byref(out)) == -1
    Q = inputs.uniform_int(10, -5, 5, 1)
    assert lib.qubo_solve_noalloc(Q.ctypes.data, 61, 0, None, ctypes.byref(out)) == -1
    assert lib.qubo_solve_noalloc(Q.ctypes.data, 10, 0, None, None) == -1
