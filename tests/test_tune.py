"""Host side of the plan tuning table and its JSON cache (no GPU needed)."""
import json

import numpy as np
import pytest

from paper_2607_04857_amd import inputs

KEY = "testdev/4cu"


@pytest.fixture()
def q():
    import paper_2607_04857_amd as q
    q.tune_clear()
    yield q
    q.tune_clear()


def _plan(q, n, **kw):
    # entries up to 5000: too large for the packed tier, so these plans are
    # the int32 walk's
    return q.plan_info(inputs.uniform_int(n, -5000, 5000, 900 + n), **kw)


def test_tuned_entry_then_packed(q):
    """A packable instance takes the tuned int32 plan one suffix bit wider
    in tier 4, with the tuned number of items."""
    q.tune_set([{"n": 30, "B": 9, "L": 12, "tier": 1, "vgpr_levels": 8}])
    d = q.plan_info(inputs.uniform_int(30, -50, 50, 930))
    assert (d["B"], d["A"], d["L"], d["tier"], d["vgpr_levels"]) == (10, 20, 11, 4, 8)
    assert d["items"] == 2 ** (21 - 12)
    # mcols 2 (B = 7) has no packed variant: the tuned int32 plan stays
    q.tune_set([{"n": 30, "B": 7, "L": 12, "tier": 2, "vgpr_levels": 12}])
    d = q.plan_info(inputs.uniform_int(30, -50, 50, 930))
    assert (d["B"], d["tier"]) == (7, 2)


def test_empty_table_gives_defaults(q):
    d = _plan(q, 30)
    assert (d["B"], d["vgpr_levels"], d["tier"]) == (10, 4, 2)
    assert q.tune_lookup(30) is None


def test_tuned_entry_drives_the_plan(q):
    q.tune_set([{"n": 30, "B": 8, "L": 12, "tier": 1, "vgpr_levels": 12}])
    d = _plan(q, 30)
    assert (d["B"], d["A"], d["L"], d["tier"], d["vgpr_levels"]) == (8, 22, 12, 1, 12)
    assert d["items"] == 2 ** (22 - 12)
    # other n and the other dtype keep the defaults
    assert _plan(q, 29)["B"] == 10
    assert q.plan_info(inputs.normal_fp32(30, 3))["B"] == 10
    # an explicit override of any walk knob bypasses the table
    assert _plan(q, 30, tier=2)["B"] == 10
    assert _plan(q, 30, B=9)["vgpr_levels"] == 12
    q.tune_clear()
    assert _plan(q, 30)["B"] == 10


def test_tuned_zero_L_keeps_default_item_size(q):
    default_L = _plan(q, 36, B=9)["L"]
    q.tune_set([{"n": 36, "B": 9, "L": 0, "tier": 2, "vgpr_levels": 8}])
    d = _plan(q, 36)
    assert (d["B"], d["L"], d["vgpr_levels"]) == (9, default_L, 8)


def test_direct_sizes_ignore_the_table(q):
    with pytest.raises(q.QuboError):
        q.tune_set([{"n": 14, "B": 6, "L": 0, "tier": 1, "vgpr_levels": 12}])
    assert _plan(q, 14)["direct"] == 1


@pytest.mark.parametrize("bad", [
    {"n": 30, "B": 5, "L": 0, "tier": 1, "vgpr_levels": 12},     # B below 6
    {"n": 30, "B": 11, "L": 0, "tier": 1, "vgpr_levels": 12},    # B above 10
    {"n": 30, "B": 8, "L": 0, "tier": 3, "vgpr_levels": 12},     # no tier 3
    {"n": 30, "B": 8, "L": 0, "tier": 2, "vgpr_levels": 6},      # G=6 needs B=10
    {"n": 30, "B": 7, "L": 0, "tier": 2, "vgpr_levels": 8},      # G=8 needs B>=9
    {"n": 30, "B": 10, "L": 21, "tier": 2, "vgpr_levels": 6},    # L > A
    {"n": 30, "B": 10, "L": 5, "tier": 2, "vgpr_levels": 6},     # L < 6
    {"n": 61, "B": 10, "L": 0, "tier": 2, "vgpr_levels": 6},     # n too large
    {"n": 16, "B": 12, "L": 0, "tier": 2, "vgpr_levels": 6},     # prefix too short
])
def test_invalid_entries_rejected_atomically(q, bad):
    good = {"n": 25, "B": 9, "L": 0, "tier": 1, "vgpr_levels": 12}
    with pytest.raises(q.QuboError) as ei:
        q.tune_set([good, bad])
    assert ei.value.status == -1
    assert q.tune_lookup(25) is None            # nothing from the call was stored


def test_save_load_roundtrip(q, tmp_path):
    ents = [{"n": 20, "B": 7, "L": 9, "tier": 1, "vgpr_levels": 12, "walk_ms": 0.25},
            {"n": 33, "dtype": "fp32", "B": 10, "L": 0, "tier": 2, "vgpr_levels": 5,
             "walk_ms": 1.5}]
    q.tune_set(ents)
    path = str(tmp_path / "tune.json")
    q.tune_save(path, KEY)
    doc = json.load(open(path))
    assert doc["format"] == "qubo-tune-1" and doc["device"] == KEY
    assert len(doc["entries"]) == 2
    q.tune_clear()
    assert q.tune_load(path, KEY) == 2
    assert q.tune_lookup(20) == {"n": 20, "dtype": "int32", "B": 7, "L": 9, "tier": 1,
                                 "vgpr_levels": 12, "walk_ms": 0.25, "scope": "single"}
    e = q.tune_lookup(33, "fp32")
    assert (e["B"], e["vgpr_levels"], e["tier"]) == (10, 5, 2)
    assert q.tune_lookup(33, "int32") is None


def test_other_device_rejected(q, tmp_path):
    q.tune_set([{"n": 20, "B": 7, "L": 9, "tier": 1, "vgpr_levels": 12}])
    path = str(tmp_path / "tune.json")
    q.tune_save(path, "gfx942/304cu")
    q.tune_clear()
    with pytest.raises(q.QuboError) as ei:
        q.tune_load(path, KEY)
    assert "gfx942/304cu" in ei.value.message
    assert q.tune_lookup(20) is None


@pytest.mark.parametrize("text", [
    "",
    "[]",
    "{\"format\": \"qubo-tune-0\", \"device\": \"%s\", \"entries\": []}" % KEY,
    "{\"format\": \"qubo-tune-1\", \"entries\": []}",
    "{\"format\": \"qubo-tune-1\", \"device\": \"%s\"}" % KEY,
    "{\"format\": \"qubo-tune-1\", \"device\": \"%s\", \"entries\": [" % KEY
    + "{\"n\": 20, \"dtype\": \"int32\", \"B\": 7, \"L\": 9, \"tier\": 1}]}",   # no vgpr_levels
    "{\"format\": \"qubo-tune-1\", \"device\": \"%s\", \"entries\": [" % KEY
    + "{\"n\": 20.5, \"dtype\": \"int32\", \"B\": 7, \"L\": 9, \"tier\": 1, \"vgpr_levels\": 12}]}",
    "{\"format\": \"qubo-tune-1\", \"device\": \"%s\", \"entries\": [" % KEY
    + "{\"n\": 20, \"dtype\": \"int8\", \"B\": 7, \"L\": 9, \"tier\": 1, \"vgpr_levels\": 12}]}",
    "{\"format\": \"qubo-tune-1\", \"device\": \"%s\", \"entries\": [" % KEY
    + "{\"n\": 20, \"dtype\": \"int32\", \"B\": 7, \"L\": 9, \"tier\": 1, \"vgpr_levels\": 12}]",
    "{\"format\": \"qubo-tune-1\", \"device\": \"%s\", \"entries\": []} x" % KEY,
])
def test_malformed_cache_rejected(q, tmp_path, text):
    path = tmp_path / "bad.json"
    path.write_text(text)
    with pytest.raises(q.QuboError) as ei:
        q.tune_load(str(path), KEY)
    assert ei.value.status == -1


def test_missing_file(q, tmp_path):
    with pytest.raises(q.QuboError):
        q.tune_load(str(tmp_path / "absent.json"), KEY)


def test_handwritten_cache_with_whitespace_and_extra_keys(q, tmp_path):
    path = tmp_path / "hand.json"
    path.write_text(json.dumps({
        "comment": "written by hand", "format": "qubo-tune-1", "device": KEY,
        "entries": [{"n": 40, "dtype": "int32", "B": 9, "L": 20, "tier": 2,
                     "vgpr_levels": 8, "note": [1, 2, {"x": None, "y": True}]}]}, indent=4))
    assert q.tune_load(str(path), KEY) == 1
    d = _plan(q, 40)
    assert (d["B"], d["L"], d["tier"], d["vgpr_levels"]) == (9, 20, 2, 8)


def test_autotune_argument_checks(q):
    for args in [(14, 20), (20, 49), (25, 20)]:
        with pytest.raises(q.QuboError) as ei:
            q.autotune(*args)
        assert ei.value.status == -1


def test_scopes_are_separate_tables(q, tmp_path):
    q.tune_set([{"n": 30, "B": 8, "L": 0, "tier": 1, "vgpr_levels": 12, "scope": "batch"}])
    assert q.tune_lookup(30) is None                       # single scope untouched
    assert q.tune_lookup(30, "int32", "batch")["B"] == 8
    assert _plan(q, 30)["B"] == 10                         # lone-solve plans ignore batch entries
    q.tune_set([{"n": 30, "B": 9, "L": 11, "tier": 2, "vgpr_levels": 8}])
    assert _plan(q, 30)["B"] == 9
    assert q.tune_lookup(30, "int32", "batch")["B"] == 8
    path = str(tmp_path / "tune.json")
    q.tune_save(path, KEY)
    doc = json.load(open(path))
    assert sorted((e["scope"], e["B"]) for e in doc["entries"]) == [("batch", 8), ("single", 9)]
    q.tune_clear()
    assert q.tune_load(path, KEY) == 2
    assert q.tune_lookup(30)["B"] == 9 and q.tune_lookup(30, "int32", "batch")["B"] == 8


def test_batch_entries_keep_the_batch_item_size(q):
    with pytest.raises(q.QuboError):
        q.tune_set([{"n": 30, "B": 8, "L": 12, "tier": 1, "vgpr_levels": 12, "scope": "batch"}])
    assert q.tune_lookup(30, "int32", "batch") is None


def test_unknown_scope_in_cache_rejected(q, tmp_path):
    path = tmp_path / "tune.json"
    path.write_text(json.dumps({"format": "qubo-tune-1", "device": KEY, "entries": [
        {"n": 30, "dtype": "int32", "B": 8, "L": 0, "tier": 1, "vgpr_levels": 12,
         "scope": "both"}]}))
    with pytest.raises(q.QuboError) as ei:
        q.tune_load(str(path), KEY)
    assert "scope" in ei.value.message


def test_shipped_cache_loads_whole(q):
    """The tuning cache shipped with the package is valid for this library: every
    entry passes the planner's checks (a stale entry would make the library
    reject the whole file and fall back to the built-in plans), both scopes
    and both dtypes are present, and an entry drives the plan it names."""
    import os
    path = os.path.join(os.path.dirname(q.__file__), "tuning", "gfx950_256cu.json")
    doc = json.load(open(path))
    assert doc["device"] == "gfx950/256cu"
    assert q.tune_load(path, "gfx950/256cu") == len(doc["entries"])
    kinds = {(e["scope"], e["dtype"]) for e in doc["entries"]}
    assert kinds == {("single", "int32"), ("single", "fp32"), ("batch", "int32"), ("batch", "fp32")}
    e = q.tune_lookup(40)
    assert e is not None
    info = q.plan_info(inputs.uniform_int(40, -10000, 10000, 40))
    assert (info["B"], info["tier"], info["vgpr_levels"]) == (e["B"], e["tier"], e["vgpr_levels"])
    # a packable instance of the same n: the entry one suffix bit wider
    info = q.plan_info(inputs.uniform_int(40, -100, 100, 40))
    assert (info["B"], info["tier"], info["vgpr_levels"]) == (e["B"] + 1, 4, e["vgpr_levels"])
