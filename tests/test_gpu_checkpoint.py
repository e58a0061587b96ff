"""Sliced, resumable solves (qubo_solve_checkpointed) against the one-shot
solve and the oracle."""
import numpy as np
import pytest

from conftest import check_fp32
from paper_2607_04857_amd import inputs

pytestmark = pytest.mark.gpu


def test_interrupted_and_resumed_equals_one_shot(tmp_path):
    import paper_2607_04857_amd as q
    Q = inputs.uniform_int(40, -10000, 10000, 3)
    whole = q.solve(Q)
    f = str(tmp_path / "n40.ckpt")
    items = q.plan_info(Q)["items"]
    per = items // 8 + 1                               # ragged last slice
    assert q.solve_checkpointed(Q, f, items_per_slice=per, max_slices=3) is None
    d = q.checkpoint_info(f)
    assert d["next_item"] == 3 * per and d["found"] == 1 and d["items"] == items
    assert q.solve_checkpointed(Q, f, items_per_slice=per, max_slices=2) is None
    assert q.checkpoint_info(f)["next_item"] == 5 * per
    r = q.solve_checkpointed(Q, f, items_per_slice=per)
    print(f"n=40 sliced: ({r.energy_i},{r.index}) whole: ({whole.energy_i},{whole.index}) "
          f"walk {r.kernel_ms:.2f} ms over 8 slices", flush=True)
    assert (r.energy_i, r.index) == (whole.energy_i, whole.index)
    assert r.states == 2 ** 40 and (r.A, r.B, r.L) == (whole.A, whole.B, whole.L)
    d = q.checkpoint_info(f)
    assert d["next_item"] == items and d["walk_ms"] == r.kernel_ms
    again = q.solve_checkpointed(Q, f, items_per_slice=per)   # finished: no device work
    assert (again.energy_i, again.index, again.kernel_ms) == (r.energy_i, r.index, r.kernel_ms)
    with pytest.raises(q.QuboError):                   # another input on the same file
        q.solve_checkpointed(inputs.uniform_int(40, -10000, 10000, 4), f)


def test_sliced_small_instances_match_oracle(tmp_path, orc):
    import paper_2607_04857_amd as q
    cases = [inputs.uniform_int(12, -100, 100, 5), inputs.uniform_int(24, -100, 100, 1),
             inputs.normal_fp32(26, 6)]
    for k, Q in enumerate(cases):
        f = str(tmp_path / f"c{k}.ckpt")
        r = q.solve_checkpointed(Q, f, items_per_slice=3)
        E, idx = orc.solve(Q, k=1)[0]
        whole = q.solve(Q)
        print(f"n={Q.shape[0]} {Q.dtype}: sliced ({r.energy_i},{r.index}) oracle ({E},{idx})",
              flush=True)
        assert (r.energy_i, r.index) == (whole.energy_i, whole.index)
        if Q.dtype == np.int32:
            assert (r.energy_i, r.index) == (E, idx)
        else:
            check_fp32(orc, Q, r, E, idx)
            assert r.energy == whole.energy


def test_planted_n46_in_slices(tmp_path, orc):
    import paper_2607_04857_amd as q
    Q, x = inputs.planted(46, -1000, 1000, 11)
    idx = int(orc.index_of(x))
    f = str(tmp_path / "p46.ckpt")
    items = q.plan_info(Q)["items"]
    assert q.solve_checkpointed(Q, f, items_per_slice=items // 4, max_slices=1) is None
    r = q.solve_checkpointed(Q, f, items_per_slice=items // 4)
    print(f"planted n=46: index {r.index} expected {idx}, E {r.energy_i}", flush=True)
    assert r.index == idx and r.energy_i == orc.energy(Q, idx)


def test_resume_keeps_the_recorded_plan(tmp_path):
    """A tuning entry installed between two calls does not change the plan of
    a solve already in progress: the resumed slices run the recorded one.
    (Entries to 10^4: the int32 walk, whose tuned B the planner takes as is.)"""
    import paper_2607_04857_amd as q
    Q = inputs.uniform_int(36, -10000, 10000, 36)
    whole = q.solve(Q)
    f = str(tmp_path / "n36.ckpt")
    items = q.plan_info(Q)["items"]
    q.tune_clear()
    try:
        assert q.solve_checkpointed(Q, f, items_per_slice=items // 4, max_slices=2) is None
        q.tune_set([{"n": 36, "B": 8, "L": 0, "tier": 1, "vgpr_levels": 12}])
        assert q.plan_info(Q)["B"] == 8                    # a fresh solve would use it
        r = q.solve_checkpointed(Q, f, items_per_slice=items // 4)
    finally:
        q.tune_clear()
    d = q.checkpoint_info(f)
    assert (r.B, d["B"], d["items"]) == (whole.B, whole.B, items)
    assert (r.energy_i, r.index) == (whole.energy_i, whole.index)


def test_packed_plan_interrupted_and_resumed(tmp_path):
    """A packable instance: the recorded plan is the packed one (tier 4, one
    suffix bit wider), and the resumed slices run it again."""
    import paper_2607_04857_amd as q
    Q = inputs.uniform_int(36, -50, 50, 37)
    whole = q.solve(Q)
    assert whole.tier == 4
    f = str(tmp_path / "p36.ckpt")
    items = q.plan_info(Q)["items"]
    per = items // 5 + 1
    assert q.solve_checkpointed(Q, f, items_per_slice=per, max_slices=2) is None
    d = q.checkpoint_info(f)
    assert (d["tier"], d["B"], d["next_item"]) == (4, whole.B, 2 * per)
    r = q.solve_checkpointed(Q, f, items_per_slice=per)
    print(f"n=36 packed sliced: ({r.energy_i},{r.index}) whole: ({whole.energy_i},{whole.index})",
          flush=True)
    assert (r.energy_i, r.index) == (whole.energy_i, whole.index)
    assert (r.tier, r.A, r.B, r.L) == (whole.tier, whole.A, whole.B, whole.L)
