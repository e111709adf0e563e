"""Host-side model of the batched task queue's persistent-launch protocol.

Rows of a queue (one per pass, in task order): level, instance, kind, tasks, dependency count, first task.
Protocol modelled: each of `blocks` resident blocks repeatedly takes the next task number from one counter,
waits until the finished-task counter of the task's instance reaches the pass's dependency count, runs the task
and then adds one to that counter; a block whose task number is past the end leaves.  Durations are one unit
per task unless `duration(kind, instance)` says otherwise.
"""
from __future__ import annotations

import heapq

import numpy as np

LEVEL, INST, KIND, TASKS, NEED, FIRST = range(6)


def static_checks(q: np.ndarray) -> list[str]:
    """Structural facts the protocol relies on; returns the violations found (empty: none)."""
    bad = []
    if len(q) == 0:
        return bad
    if np.any(np.diff(q[:, LEVEL]) < 0):
        bad.append("pass levels decrease along the queue")
    ends = q[:, FIRST] + q[:, TASKS]
    if np.any(q[1:, FIRST] != ends[:-1]) or q[0, FIRST] != 0:
        bad.append("passes do not tile the task range")
    seen: dict[int, int] = {}
    last_end: dict[int, int] = {}
    for r in q:
        i = int(r[INST])
        if int(r[NEED]) != seen.get(i, 0):
            bad.append(f"pass at task {int(r[FIRST])}: dependency count {int(r[NEED])} != {seen.get(i, 0)} "
                       f"earlier tasks of instance {i}")
        if last_end.get(i, 0) > int(r[FIRST]):
            bad.append(f"pass at task {int(r[FIRST])} precedes a pass it depends on")
        seen[i] = seen.get(i, 0) + int(r[TASKS])
        last_end[i] = int(r[FIRST] + r[TASKS])
    return bad


def simulate(q: np.ndarray, blocks: int, duration=None) -> dict:
    """Event simulation of the protocol.  Returns finished (every task ran and every block left),
    deadlock (blocks still waiting with nothing running), makespan, the largest number of blocks waiting
    at once, and per-instance finished counts against the instance's task totals."""
    n_tasks = int(q[:, TASKS].sum()) if len(q) else 0
    firsts = q[:, FIRST] if len(q) else np.zeros(0, dtype=np.int64)
    totals: dict[int, int] = {}
    for r in q:
        totals[int(r[INST])] = totals.get(int(r[INST]), 0) + int(r[TASKS])
    done: dict[int, int] = {i: 0 for i in totals}
    waiting: dict[int, list] = {}  # instance -> heap of (need, block, task, pass)
    events: list = []  # (time, seq, block, pass) task completions
    nxt = 0
    seq = 0
    ran = 0
    max_wait = 0
    n_wait = 0
    active = blocks

    def dur(pi):
        return 1.0 if duration is None else float(duration(int(q[pi, KIND]), int(q[pi, INST])))

    def take(block, now):
        nonlocal nxt, seq, active, n_wait, max_wait
        t = nxt
        nxt += 1
        if t >= n_tasks:
            active -= 1
            return
        pi = int(np.searchsorted(firsts, t, side="right") - 1)
        i, need = int(q[pi, INST]), int(q[pi, NEED])
        if done[i] >= need:
            heapq.heappush(events, (now + dur(pi), seq, block, pi))
            seq += 1
        else:
            heapq.heappush(waiting.setdefault(i, []), (need, block, t, pi))
            n_wait += 1
            max_wait = max(max_wait, n_wait)

    now = 0.0
    for b in range(blocks):
        take(b, now)
    while events:
        now, _, b, pi = heapq.heappop(events)
        ran += 1
        i = int(q[pi, INST])
        done[i] += 1
        w = waiting.get(i, [])
        while w and w[0][0] <= done[i]:
            _, wb, _, wpi = heapq.heappop(w)
            n_wait -= 1
            heapq.heappush(events, (now + dur(wpi), seq, wb, wpi))
            seq += 1
        take(b, now)
    return {"finished": ran == n_tasks and active == 0 and n_wait == 0,
            "deadlock": n_wait > 0,
            "makespan": now,
            "max_waiting": max_wait,
            "tasks_run": ran,
            "counts_match": all(done[i] == totals[i] for i in totals)}


def level_makespan(q: np.ndarray, blocks: int) -> int:
    """Unit-duration makespan of the level-synchronous schedule: each level's tasks spread over the blocks,
    the next level after all of them."""
    tot = 0
    for lv in np.unique(q[:, LEVEL]):
        k = int(q[q[:, LEVEL] == lv, TASKS].sum())
        tot += -(-k // blocks)
    return tot
