"""Pins for the host-side model of the batched task queue (tests/queue_sim.py): closed-form makespans,
and planted queue mistakes (a wrong dependency count, a dependency placed after its dependant) that the
structural checks and the event simulation must catch."""
import numpy as np

import queue_sim as qs


def _queue(inst_passes, order=None):
    """inst_passes[i] = task counts of instance i's passes; queue level by level (instances in `order`)."""
    n = len(inst_passes)
    order = list(range(n)) if order is None else order
    rows, first, seen = [], 0, [0] * n
    for lv in range(max(len(p) for p in inst_passes)):
        for i in order:
            if lv < len(inst_passes[i]):
                k = inst_passes[i][lv]
                rows.append([lv, i, 0, k, seen[i], first])
                first += k
                seen[i] += k
    return np.array(rows, dtype=np.int64)


def test_single_chain_makespan_closed_form():
    passes = [5, 1, 9, 3, 16]
    q = _queue([passes])
    assert qs.static_checks(q) == []
    for B in (1, 2, 4, 7, 64):
        r = qs.simulate(q, B)
        assert r["finished"] and r["counts_match"] and not r["deadlock"]
        assert r["makespan"] == sum(-(-k // B) for k in passes) == qs.level_makespan(q, B)


def test_many_instances_finish_and_count():
    rng = np.random.default_rng(0)
    inst = [list(rng.integers(1, 12, size=rng.integers(3, 30))) for _ in range(40)]
    q = _queue(inst, order=list(rng.permutation(40)))
    assert qs.static_checks(q) == []
    for B in (1, 3, 16, 200):
        r = qs.simulate(q, B, duration=lambda kind, i: 1 + (i % 5))
        assert r["finished"] and r["counts_match"] and r["tasks_run"] == int(q[:, qs.TASKS].sum())
    # one block runs the queue in order: makespan = total duration
    r = qs.simulate(q, 1)
    assert r["makespan"] == int(q[:, qs.TASKS].sum()) and r["max_waiting"] == 0


def test_planted_wrong_dependency_count_is_caught():
    q = _queue([[3, 2, 4], [1, 1, 1]])
    bad = q.copy()
    row = np.where((bad[:, qs.INST] == 0) & (bad[:, qs.LEVEL] == 2))[0][0]
    bad[row, qs.NEED] += 1  # waits for one task more than instance 0 ever finishes before it
    assert any("dependency count" in m for m in qs.static_checks(bad))
    r = qs.simulate(bad, 4)
    assert r["deadlock"] and not r["finished"]


def test_planted_out_of_order_dependency_is_caught():
    q = _queue([[2, 2], [1, 1]])
    # move instance 0's second pass ahead of its first: the queue no longer lists dependencies first
    a = np.where((q[:, qs.INST] == 0) & (q[:, qs.LEVEL] == 0))[0][0]
    b = np.where((q[:, qs.INST] == 0) & (q[:, qs.LEVEL] == 1))[0][0]
    rows = list(q)
    rows[a], rows[b] = rows[b].copy(), rows[a].copy()
    first = 0
    for r in rows:
        r[qs.FIRST] = first
        first += r[qs.TASKS]
    bad = np.array(rows)
    assert qs.static_checks(bad)
    # a single block takes the dependant first and waits for ever
    assert qs.simulate(bad, 1)["deadlock"]
