"""Batched LUCJ energy + adjoint gradient: many sectors run together, one launch per pass kind of each level
(the default) or one cooperative launch.

Parity: every instance against the oracle's energy and adjoint gradient
(1e-12 (complex128) / 1e-5 (complex64) on energies relative to max(1, |E|) and
on gradients relative to max(1, |g|_inf)), against the single-instance GPU
path, and for the 256-instance batched workload against stored oracle
results (tests/golden/batched_config4.txt).
"""
import os

import numpy as np
import pytest
import torch

from oracle import lucj as ol
from paper_2605_03123_amd import synth
from errlog import record

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "batched_config4.txt")
TOL = {torch.complex128: (1e-12, 1e-12), torch.complex64: (1e-5, 1e-5)}


@pytest.fixture(scope="module")
def ffx():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_2605_03123_amd import ffx as mod
    return mod


def _instances(sectors, seed, n_reps=2):
    out = []
    for k, (norb, nelec) in enumerate(sectors):
        r = synth.rng([seed, k])
        out.append((norb, nelec, synth.lucj_params(r, norb, n_reps), synth.df_hamiltonian(r, norb, norb)))
    return out


def _check(e, g, e_ref, g_ref, dtype, name="batched"):
    te, tg = TOL[dtype]
    assert record(name, dtype, "energy_rel", abs(e - e_ref) / max(1.0, abs(e_ref)), te) <= te
    err = np.max(np.abs(g - g_ref)) / max(1.0, np.max(np.abs(g_ref)))
    assert record(name, dtype, "grad_rel", err, tg) <= tg


SMALL = {
    torch.complex128: [(6, (3, 3)), (7, (3, 4)), (8, (4, 4)), (6, (2, 3)), (8, (3, 3)), (7, (2, 2))],
    torch.complex64: [(8, (4, 4)), (8, (3, 3)), (8, (3, 4)), (9, (4, 4)), (8, (2, 5))],
}


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_batched_small_vs_oracle(ffx, dtype):
    inst = _instances(SMALL[dtype], seed=40)
    b = ffx.Batch([(n, ne) for n, ne, _, _ in inst], dtype=dtype)
    print(f"batched launch: {len(inst)} sectors {dtype} {b.info()}", flush=True)
    e, g = b.lucj_energy_grad([p for *_, p, _ in inst], [h for *_, h in inst], 2)
    print("batched launch done", flush=True)
    for i, (norb, nelec, p, ham) in enumerate(inst):
        eo, go = ol.grad_adjoint(p, ham, norb, nelec, 2)
        _check(e[i], g[i], float(np.real(eo)), go, dtype)


def test_batched_matches_single_instance(ffx):
    dtype = torch.complex128
    sectors = [(8, (4, 4)), (10, (5, 5)), (10, (4, 4)), (8, (3, 3)), (10, (4, 5)), (8, (4, 4)), (9, (4, 4))]
    inst = _instances(sectors, seed=41, n_reps=3)
    b = ffx.Batch(sectors, dtype=dtype)
    e, g = b.lucj_energy_grad([p for *_, p, _ in inst], [h for *_, h in inst], 3)
    for i, (norb, nelec, p, ham) in enumerate(inst):
        e1, g1 = ffx.lucj_energy_grad(p, ham, norb, nelec, 3, dtype=dtype)
        _check(e[i], g[i], e1, g1, dtype)


def test_batched_repeatable_and_tuned(ffx):
    dtype = torch.complex128
    sectors = [(8, (4, 4)), (10, (5, 5)), (8, (3, 3))]
    inst = _instances(sectors, seed=42)
    args = ([p for *_, p, _ in inst], [h for *_, h in inst], 2)
    b = ffx.Batch(sectors, dtype=dtype)
    e0, g0 = b.lucj_energy_grad(*args)
    e1, g1 = b.lucj_energy_grad(*args)
    assert np.array_equal(e0, e1) and all(np.array_equal(x, y) for x, y in zip(g0, g1))
    t, r = b.tune(*args)
    assert t > 0 and r > 0 and b.info()["target_elems"] == t
    e2, g2 = b.lucj_energy_grad(*args)
    for i in range(len(sectors)):
        _check(e2[i], g2[i], e0[i], g0[i], dtype)


def test_batched_errors(ffx):
    with pytest.raises(ffx.FFXError):
        ffx.Batch([(5, (2, 2))], dtype=torch.complex64)  # below the register window
    b = ffx.Batch([(8, (4, 4))], dtype=torch.complex64)
    inst = _instances([(8, (4, 4))], seed=43)
    with pytest.raises(ValueError):
        b.lucj_energy_grad([inst[0][2][:-1]], [inst[0][3]], 2)


def _golden():
    out = {}
    with open(GOLDEN) as f:
        lines = [ln.split() for ln in f if not ln.startswith("#")]
    for head, grad in zip(lines[0::2], lines[1::2]):
        out[int(head[1])] = (float(head[5]), np.array([float(v) for v in grad]))
    return out


@pytest.mark.skipif(not os.path.exists(GOLDEN), reason="golden file not generated")
def test_batched_config4(ffx):
    # 256 instances, norb in {8, 10, 12}, in both precisions
    w = synth.workload_batched(256, seed=0, n_reps=2)
    sectors = [(x.norb, x.nelec) for x in w]
    args = ([x.data["params"] for x in w], [x.data["ham"] for x in w], 2)
    gold = _golden()
    res = {}
    for dtype in (torch.complex64, torch.complex128):
        b = ffx.Batch(sectors, dtype=dtype)
        print(f"batched launch: 256 sectors {dtype} {b.info()}", flush=True)
        e, g = b.lucj_energy_grad(*args)
        print("batched launch done", flush=True)
        for i, (eo, go) in gold.items():
            _check(e[i], g[i], eo, go, dtype, "batched_config4_vs_oracle")
        res[dtype] = (e, g)
    e64, g64 = res[torch.complex64]
    e128, g128 = res[torch.complex128]
    for i in range(len(w)):
        _check(e64[i], g64[i], e128[i], g128[i], torch.complex64, "batched_config4_c64_vs_c128")


def test_batched_single_cooperative_launch(ffx):
    """The whole batch as one cooperative launch (grid barrier between pass levels): energies and gradients
    identical to the launches per pass kind of each level, in both precisions, over two calls in a row."""
    w = synth.workload_batched(64, seed=3, n_reps=2)
    sectors = [(x.norb, x.nelec) for x in w]
    args = ([x.data["params"] for x in w], [x.data["ham"] for x in w], 2)
    for dtype in (torch.complex64, torch.complex128):
        b = ffx.Batch(sectors, dtype=dtype)
        b.single_launch(False)
        e0, g0 = b.lucj_energy_grad(*args)
        assert b.timing()["launches"] > 1
        b.single_launch(True)
        print(f"cooperative batched launch: 64 sectors {dtype}", flush=True)
        for _ in range(2):
            e1, g1 = b.lucj_energy_grad(*args)
            assert b.timing()["launches"] == 1
            np.testing.assert_array_equal(e1, e0)
            for a, c in zip(g1, g0):
                np.testing.assert_array_equal(a, c)
        b.single_launch(False)
        e2, _ = b.lucj_energy_grad(*args)
        np.testing.assert_array_equal(e2, e0)


def test_batched_queue_protocol(ffx):
    """The task queue of the 256-sector workload, as the library builds it (nothing launched), run through
    the host model of the persistent launch's protocol at the launch's resident block count: the queue lists
    every pass after the passes it depends on, each dependency count equals the instance's earlier tasks, the
    model finishes without a stuck wait and counts every task of every instance."""
    import queue_sim as qs
    w = synth.workload_batched(256, seed=0, n_reps=2)
    b = ffx.Batch([(x.norb, x.nelec) for x in w], dtype=torch.complex64)
    q = b.queue([x.data["params"] for x in w], [x.data["ham"] for x in w], 2)
    blocks = b.info()["blocks"]
    assert len(q) and blocks > 0
    assert qs.static_checks(q) == []
    r = qs.simulate(q, blocks)
    assert r["finished"] and r["counts_match"] and not r["deadlock"], r
    n_tasks, levels = int(q[:, qs.TASKS].sum()), len(np.unique(q[:, qs.LEVEL]))
    print(f"batched queue: {len(q)} passes, {n_tasks} tasks, {levels} levels, {blocks} resident blocks; "
          f"unit-time makespan {r['makespan']:.0f} (level-synchronous {qs.level_makespan(q, blocks)}), "
          f"at most {r['max_waiting']} blocks waiting", flush=True)


@pytest.mark.skip(reason="the single persistent launch (task queue with per-instance dependency counters) is "
                         "switched off: its GPU runs did not complete, and the cause is not established (the "
                         "queue protocol is shown deadlock-free on the host by test_batched_queue_protocol); "
                         "batches run as one cooperative launch or one launch per pass level")
def test_batched_persistent_single_launch(ffx):
    """The persistent launch gives the per-level launches' energies and gradients bit for bit, in both
    precisions, over two calls in a row, and ends in one launch."""
    w = synth.workload_batched(16, seed=5, n_reps=1)
    sectors = [(x.norb, x.nelec) for x in w]
    args = ([x.data["params"] for x in w], [x.data["ham"] for x in w], 1)
    for dtype in (torch.complex64, torch.complex128):
        b = ffx.Batch(sectors, dtype=dtype)
        b.single_launch(False)
        e0, g0 = b.lucj_energy_grad(*args)
        b.persistent(True)
        for _ in range(2):
            e1, g1 = b.lucj_energy_grad(*args)
            assert b.timing()["launches"] == 1
            np.testing.assert_array_equal(e1, e0)
            for a, c in zip(g1, g0):
                np.testing.assert_array_equal(a, c)
        b.persistent(False)
