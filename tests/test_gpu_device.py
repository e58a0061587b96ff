"""GPU: qubo_solve_device on matrices held in device memory.

The fold, the int32 exactness proof and the float32 scaling run in a device
kernel there, so every field of the result must equal qubo_solve's on a host
copy of the same matrix (same T, p, tol and answer), and the answer must be
the oracle's.  Input errors come back as the host planner's statuses.  The
device plan is made from n and the dtype alone, so it never takes the
packed tier (which depends on the values); the int32 inputs compared here
have entries large enough that the host plan does not take it either.
"""
import json
import os

import numpy as np
import pytest

from conftest import GOLDEN, check_fp32
from paper_2607_04857_amd import inputs

pytestmark = pytest.mark.gpu

FIELDS = ("energy_i", "energy", "index", "tol", "p", "A", "B", "L", "tier", "vgpr_levels", "states")


@pytest.fixture(scope="module")
def env():
    import torch   # torch's HIP runtime first, then the library
    import paper_2607_04857_amd as q
    q.lib()
    return q, torch


def _same(a, b):
    for f in FIELDS:
        assert getattr(a, f) == getattr(b, f), (f, a, b)


@pytest.mark.parametrize("n,seed", [(1, 1), (9, 2), (14, 3), (15, 4), (20, 5), (26, 6), (33, 7)])
def test_int32_equals_host_and_oracle(env, orc, n, seed):
    q, torch = env
    Q = inputs.uniform_int(n, -10000, 10000, 900 + seed)
    dev = q.solve_device(torch.from_numpy(Q).cuda())
    host = q.solve(Q)
    print(f"n={n} device ({dev.energy_i}, {dev.index}) host ({host.energy_i}, {host.index})",
          flush=True)
    _same(dev, host)
    if n <= 26:
        assert (dev.energy_i, dev.index) == orc.solve(Q, k=1)[0]


@pytest.mark.parametrize("n,seed", [(7, 1), (18, 2), (24, 3), (31, 4)])
def test_fp32_equals_host_and_oracle(env, orc, n, seed):
    q, torch = env
    Q = inputs.normal_fp32(n, 950 + seed)
    dev = q.solve_device(torch.from_numpy(Q).cuda())
    host = q.solve(Q)
    print(f"n={n} device ({dev.energy}, {dev.index}, p={dev.p}) host ({host.energy}, "
          f"{host.index}, p={host.p})", flush=True)
    _same(dev, host)
    if n <= 24:
        E, idx = orc.solve(Q, k=1)[0]
        check_fp32(orc, Q, dev, E, idx)


def test_lower_triangle_is_folded(env):
    """A full (not upper-triangular) matrix: the device fold adds Q_ji to Q_ij."""
    q, torch = env
    rng = np.random.default_rng(5)
    Q = rng.integers(-5000, 5001, (22, 22)).astype(np.int32)
    _same(q.solve_device(torch.from_numpy(Q).cuda()), q.solve(Q))
    Qf = rng.standard_normal((22, 22)).astype(np.float32)
    _same(q.solve_device(torch.from_numpy(Qf).cuda()), q.solve(Qf))


@pytest.mark.parametrize("kind,n,k", [("int", 12, 16), ("int", 26, 64), ("fp32", 23, 32)])
def test_topk_equals_host(env, kind, n, k):
    q, torch = env
    Q = inputs.uniform_int(n, -10000, 10000, 970 + n) if kind == "int" else inputs.normal_fp32(n, 970 + n)
    dev, dl = q.solve_device(torch.from_numpy(Q).cuda(), k=k)
    host, hl = q.solve(Q, k=k)
    _same(dev, host)
    assert dl == hl


def test_headline_instance_equals_oracle(env):
    """The n = 44 headline instance from device memory equals the stored
    oracle answer over all 2^44 states."""
    q, torch = env
    with open(os.path.join(GOLDEN, "oracle_results.json")) as f:
        e = json.load(f)["n44_int_u10000_s4"]
    Q = inputs.uniform_int(**e["kwargs"])
    dev = q.solve_device(torch.from_numpy(Q).cuda())
    print("device44", dev.energy_i, dev.index, f"{dev.kernel_ms:.1f} ms", flush=True)
    assert [dev.energy_i, dev.index] == e["best"]


def test_input_errors_and_recovery(env):
    q, torch = env
    big = np.zeros((16, 16), dtype=np.int32)
    big[0, 1] = 2 ** 29
    big[1, 0] = 2 ** 29          # folded: |T_01| = 2^30 > 2^30 - 1
    with pytest.raises(q.QuboError) as ei:
        q.solve_device(torch.from_numpy(big).cuda())
    assert ei.value.status == -2          # QUBO_EOVERFLOW
    with pytest.raises(q.QuboError) as eh:
        q.solve(big)
    assert eh.value.status == -2
    nan = inputs.normal_fp32(20, 3)
    nan[3, 7] = np.nan
    with pytest.raises(q.QuboError) as en:
        q.solve_device(torch.from_numpy(nan).cuda())
    assert en.value.status == -3          # QUBO_ENONFINITE
    inf = inputs.normal_fp32(10, 4)
    inf[9, 2] = np.inf           # lower triangle, direct path
    with pytest.raises(q.QuboError) as ef:
        q.solve_device(torch.from_numpy(inf).cuda())
    assert ef.value.status == -3
    # (entries to 10^4: a host solve of smaller ones could take the packed
    # tier, which the shape-only device plan does not)
    ok = inputs.uniform_int(24, -10000, 10000, 11)
    _same(q.solve_device(torch.from_numpy(ok).cuda()), q.solve(ok))


def test_stream_order(env):
    """The matrix is written by a kernel on a side stream and solved on that
    stream with no synchronisation in between."""
    q, torch = env
    Q = inputs.uniform_int(28, -10000, 10000, 77)
    src = torch.from_numpy(Q).cuda()
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        dst = torch.zeros_like(src)
        dst.copy_(src)
        dst.mul_(1)
    dev = q.solve_device(dst, stream=s)
    _same(dev, q.solve(Q))
