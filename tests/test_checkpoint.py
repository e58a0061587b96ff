"""Checkpoint files of sliced solves: host-side reading, validation and resume
of a finished checkpoint (no GPU work)."""
import ctypes

import numpy as np
import pytest

from paper_2607_04857_amd import inputs


def fnv1a64(Q):
    """FNV-1a (64 bit) over n, the dtype code and the raw n*n input words."""
    Q = np.ascontiguousarray(Q)
    code = 1 if Q.dtype == np.float32 else 0
    data = np.array([Q.shape[0], code], dtype="<u4").tobytes() + Q.astype(Q.dtype.newbyteorder("<")).tobytes()
    h = 0xcbf29ce484222325
    for b in data:
        h ^= b
        h = (h * 0x100000001b3) & 0xFFFFFFFFFFFFFFFF
    return h


def write(path, n=20, dtype=0, qhash=0x1234, plan=(10, 10, 5, 2, 12), items=32, next_item=8,
          found=1, energy_i=-77, energy=-77.0, index=5, p=0, tol=0.0, walk_ms=1.5, extra=""):
    path.write_text(
        f"qubo-checkpoint 1\nn {n}\ndtype {dtype}\nqhash {qhash:016x}\n"
        f"plan {' '.join(str(v) for v in plan)}\nitems {items}\nnext_item {next_item}\n"
        f"found {found}\nenergy_i {energy_i}\nenergy {energy!r}\nindex {index}\np {p}\n"
        f"tol {tol!r}\nwalk_ms {walk_ms!r}\n{extra}")


def test_info_reads_every_field(tmp_path):
    import paper_2607_04857_amd as q
    f = tmp_path / "c.txt"
    write(f)
    d = q.checkpoint_info(str(f))
    assert (d["n"], d["dtype"], d["q_hash"]) == (20, "int32", 0x1234)
    assert (d["A"], d["B"], d["L"], d["tier"], d["vgpr_levels"]) == (10, 10, 5, 2, 12)
    assert (d["items"], d["next_item"], d["found"]) == (32, 8, 1)
    assert d["best"] == (-77, -77.0, 5) and d["walk_ms"] == 1.5


@pytest.mark.parametrize("bad", [
    dict(extra="junk\n"), dict(next_item=33), dict(found=0), dict(n=0), dict(n=61),
    dict(dtype=2), dict(index=1 << 20), dict(plan=(9, 10, 5, 2, 12)), dict(walk_ms=-1.0),
])
def test_malformed_checkpoints_are_rejected(tmp_path, bad):
    import paper_2607_04857_amd as q
    f = tmp_path / "c.txt"
    write(f, **bad)
    with pytest.raises(q.QuboError) as e:
        q.checkpoint_info(str(f))
    assert e.value.status == -1 and "malformed" in e.value.message


def test_truncated_and_missing_files(tmp_path):
    import paper_2607_04857_amd as q
    f = tmp_path / "c.txt"
    write(f)
    f.write_text("\n".join(f.read_text().splitlines()[:7]) + "\n")
    with pytest.raises(q.QuboError):
        q.checkpoint_info(str(f))
    f.write_text("qubo-checkpoint 2\n")
    with pytest.raises(q.QuboError):
        q.checkpoint_info(str(f))
    with pytest.raises(q.QuboError) as e:
        q.checkpoint_info(str(tmp_path / "absent.txt"))
    assert "no checkpoint" in e.value.message


def test_checkpoint_of_another_input_is_rejected_before_any_device_work(tmp_path):
    import paper_2607_04857_amd as q
    Q = inputs.uniform_int(20, -100, 100, 1)
    f = tmp_path / "c.txt"
    write(f, qhash=fnv1a64(Q) ^ 1)
    with pytest.raises(q.QuboError) as e:
        q.solve_checkpointed(Q, str(f))
    assert "another input" in e.value.message
    plan = q.plan_info(Q)
    write(f, qhash=fnv1a64(Q), plan=(plan["A"], plan["B"], plan["L"], plan["tier"],
                                     plan["vgpr_levels"]))
    with pytest.raises(q.QuboError) as e:             # contradicting override
        q.solve_checkpointed(Q, str(f), B=plan["B"] - 1)
    assert "another plan" in e.value.message


def test_finished_checkpoint_returns_its_result_without_device_work(tmp_path):
    import paper_2607_04857_amd as q
    for Q in (inputs.uniform_int(20, -100, 100, 2), inputs.normal_fp32(18, 3)):
        plan = q.plan_info(Q)
        f = tmp_path / "done.txt"
        write(f, n=Q.shape[0], dtype=1 if Q.dtype == np.float32 else 0, qhash=fnv1a64(Q),
              plan=(plan["A"], plan["B"], plan["L"], plan["tier"], plan["vgpr_levels"]),
              items=plan["items"], next_item=plan["items"], energy_i=-5, energy=-5.25, index=9,
              p=plan["p"], tol=0.5, walk_ms=2.0)
        r = q.solve_checkpointed(Q, str(f))
        assert (r.energy_i, r.energy, r.index, r.tol, r.kernel_ms) == (-5, -5.25, 9, 0.5, 2.0)
        assert r.states == 2 ** Q.shape[0] and (r.A, r.B, r.L) == (plan["A"], plan["B"], plan["L"])


def test_argument_checks(tmp_path):
    import paper_2607_04857_amd as q
    lib = q.lib()
    Q = inputs.uniform_int(20, -100, 100, 1)
    out = q._Result()
    assert lib.qubo_solve_checkpointed(Q.ctypes.data, 20, 0, None, 0, 0, None,
                                       ctypes.byref(out)) == -1
    assert lib.qubo_solve_checkpointed(Q.ctypes.data, 20, 0, None, 0, -1,
                                       str(tmp_path / "x").encode(), ctypes.byref(out)) == -1
    opt = q._options(item_first=1, item_count=1)
    assert lib.qubo_solve_checkpointed(Q.ctypes.data, 20, 0, ctypes.byref(opt), 0, 0,
                                       str(tmp_path / "x").encode(), ctypes.byref(out)) == -1
    assert lib.qubo_solve_checkpointed(Q.ctypes.data, 0, 0, None, 0, 0,
                                       str(tmp_path / "x").encode(), ctypes.byref(out)) == -1
    assert not (tmp_path / "x").exists()
