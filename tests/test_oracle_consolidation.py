"""Pins for the consolidation bookkeeping oracle against the paper's worked
example (Sec. IV.A, Fig. 2) and the Sec. IV.E buffer-size and KC_X rules, stored
as cited fixtures under tests/golden/."""
import os

import numpy as np

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def read_fixture(name):
    rows = {}
    lines = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            key, *vals = line.split()
            lines.append((key, [int(v) for v in vals]))
            rows[key] = [int(v) for v in vals]
    return rows, lines


def test_fig2_two_children_become_one_consolidated_child():
    rows, _ = read_fixture("fig2_consolidation.txt")
    work = np.array(rows["work"])
    t = rows["threshold"][0]
    # one scope covering all threads (the block of Fig. 2 / the grid)
    plan = oracle.consolidation_plan(work, t, len(work))
    assert plan["basic_launches"] == rows["basic_launches"][0]
    assert plan["dispatches"] == rows["consolidated_dispatches"][0]
    assert plan["items"] == rows["consolidated_items"][0]
    assert plan["total_work"] == rows["consolidated_work"][0]
    # scope of one thread is the basic template: one dispatch per heavy thread
    plan1 = oracle.consolidation_plan(work, t, 1)
    assert plan1["dispatches"] == plan1["basic_launches"] == 2
    assert oracle.count_heavy(work, t) == 2


def test_scopes_bound_the_reduction():
    """Warp-level consolidation reduces launches by at most the scope width (Sec. IV.B)."""
    rng = np.random.default_rng(2)
    work = rng.integers(0, 200, size=10000)
    t = 100
    base = oracle.consolidation_plan(work, t, 1)["dispatches"]
    prev = base
    for scope in (32, 64, 256, 1024, len(work)):
        plan = oracle.consolidation_plan(work, t, scope)
        assert plan["items"] == base
        assert plan["dispatches"] >= -(-base // scope)
        assert plan["dispatches"] <= -(-len(work) // scope)
        assert plan["dispatches"] <= prev
        prev = plan["dispatches"]
    assert oracle.consolidation_plan(work, t, len(work))["dispatches"] == 1
    assert oracle.consolidation_plan(np.zeros(10), 0, 4)["dispatches"] == 0


def test_per_buffer_size_and_kc_config():
    _, lines = read_fixture("buffer_and_kc.txt")
    for key, v in lines:
        if key == "pbs":
            assert oracle.per_buffer_size(v[0], v[1], v[2]) == v[3]
        elif key == "kc":
            assert oracle.kc_config(v[0], v[1], v[2]) == (v[3], v[4])
