"""The committed schedule table (paper_2306_08623_amd/schedules.json) and
the autotuner's class boundaries, on the CPU: every entry is a valid
(kind, r, s) with a grid the library accepts, the classes of one kind and
pair cover ascending n_r ranges, and the boundaries sit between the
measured sizes."""
from __future__ import annotations

import json
import os

from paper_2306_08623_amd import autotune, nucleus

U64_MAX = (1 << 64) - 1


def test_table_entries_are_valid_and_ordered():
    path = nucleus.SCHEDULES_PATH
    assert os.path.exists(path)
    with open(path) as f:
        table = json.load(f)
    entries = table["entries"]
    assert entries, "empty schedule table"
    assert nucleus.load_schedules() == entries
    groups = {}
    for e in entries:
        assert e["kind"] in (nucleus.ND_SCHED_SINGLE, nucleus.ND_SCHED_BATCH)
        assert 1 <= e["r"] < e["s"] <= 7
        assert 0 <= e["peel_blocks"] <= 2048
        assert 0 < e["n_r_max"] <= U64_MAX
        groups.setdefault((e["kind"], e["r"], e["s"]), []).append(e["n_r_max"])
    for key, ends in groups.items():
        assert ends == sorted(ends) and len(set(ends)) == len(ends), key
    # batch classes cover every size; the measured timings are kept beside them
    for (kind, r, s), ends in groups.items():
        if kind == nucleus.ND_SCHED_BATCH:
            assert ends[-1] == U64_MAX, (r, s)
    assert all(t["seconds"] > 0 for t in table["timings"])


def test_class_boundaries_are_geometric_midpoints():
    classes = [(100, 64), (10_000, 256), (1_000_000, 0)]
    ent = autotune._classes_to_entries(nucleus.ND_SCHED_BATCH, 3, 4, classes)
    assert [e["peel_blocks"] for e in ent] == [64, 256, 0]
    assert ent[0]["n_r_max"] == 1000 and ent[1]["n_r_max"] == 100_000
    assert ent[2]["n_r_max"] == U64_MAX
    for e in ent:
        assert (e["kind"], e["r"], e["s"]) == (nucleus.ND_SCHED_BATCH, 3, 4)
