"""Error paths under injected allocation failures.

With FFX_FAULT=alloc:<k>, the k-th allocation the library makes (device or pinned host memory) fails as if the
runtime had refused it.  For each k up to the first that lets the call through, the call must return FFX_ENOMEM
with a message, leave the plan (or batch) usable, and the next call without the hook must give the same result
as a run that never failed.  Covers plan creation, the lazily allocated buffers of the LUCJ and DF-chain
gradients (temporary states, result block, table arena, rank tables, transition-matrix string tables) and the
batched call (scratch, arena, upload buffers, counters)."""
import contextlib
import os

import numpy as np
import pytest
import torch

from oracle import gates as og
from paper_2605_03123_amd import synth

pytestmark = pytest.mark.gpu
ENOMEM = -3


@pytest.fixture(scope="module")
def ffx():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_2605_03123_amd import ffx as mod
    return mod


@contextlib.contextmanager
def fault(k):
    os.environ["FFX_FAULT"] = f"alloc:{k}"
    try:
        yield
    finally:
        os.environ.pop("FFX_FAULT", None)


def _until_success(ffx, call, max_k=400):
    """Runs call() with the k-th allocation failing, k = 1, 2, ... until it succeeds; returns (k, result).
    After each failure, checks the error code and message."""
    for k in range(1, max_k):
        with fault(k):
            try:
                res = call()
            except ffx.FFXError as e:
                assert e.code == ENOMEM, (k, str(e))
                assert "alloc" in str(e) or "hipMalloc" in str(e), str(e)
                continue
        return k, res
    raise AssertionError("the call never got through")


def _sampled(ffx, call, ks):
    """Runs call() with the k-th allocation failing for each k in ks (each must fail cleanly or go
    through), then once without the hook; returns that last result."""
    for k in ks:
        with fault(k):
            try:
                res = call()
                del res
            except ffx.FFXError as e:
                assert e.code == ENOMEM, (k, str(e))
    return call()


def test_plan_creation_at_every_allocation(ffx):
    norb, nelec = 8, (4, 3)
    r = synth.rng(4)
    vec = synth.random_state(r, synth.dim(norb, 4), synth.dim(norb, 3))
    U = synth.random_unitary(r, norb)
    vd = torch.from_numpy(vec).cuda()

    def rotate(plan):
        out = ffx.apply_orbital_rotation(vd, U, norb, nelec, plan=plan)
        np.testing.assert_allclose(out.cpu().numpy(), og.apply_orbital_rotation(vec, U, norb, nelec), atol=1e-12)

    # first use loads the library's code objects onto the device: before the baseline
    warm = ffx.Plan(norb, nelec, torch.complex128)
    rotate(warm)
    del warm
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    print("fault injection: plan creation", flush=True)
    k, plan = _until_success(ffx, lambda: ffx.Plan(norb, nelec, torch.complex128))
    assert k > 5, k  # plan creation makes several allocations, each of which failed once
    rotate(plan)
    del plan
    torch.cuda.synchronize()
    # the failed creations released what they had allocated (pinned ring and device tables alike)
    assert torch.cuda.mem_get_info()[0] > free0 - (64 << 20)


def test_gradients_after_failed_lazy_allocations(ffx):
    norb, nelec = 6, (3, 2)
    r = synth.rng(8)
    params = synth.lucj_params(r, norb, 2)
    ham = synth.df_hamiltonian(r, norb, 3)
    obs = synth.df_hamiltonian(r, norb, 2)
    vec0 = torch.from_numpy(synth.random_state(r, synth.dim(norb, 3), synth.dim(norb, 2))).cuda()
    ref_plan = ffx.Plan(norb, nelec, torch.complex128)
    e_ref, g_ref = ffx.lucj_energy_grad(params, ham, norb, nelec, 2, plan=ref_plan)
    c_ref, cg_ref = ffx.df_chain_energy_grad(vec0, ham, obs, 0.1, 2, norb, nelec, plan=ref_plan)
    print("fault injection: LUCJ and DF-chain gradients on a fresh plan", flush=True)
    plan = ffx.Plan(norb, nelec, torch.complex128)
    k1, (e, g) = _until_success(ffx, lambda: ffx.lucj_energy_grad(params, ham, norb, nelec, 2, plan=plan))
    assert k1 > 1  # the first gradient call allocates lazily
    assert e == e_ref and np.array_equal(g, g_ref)
    k2, (c, cg) = _until_success(ffx, lambda: ffx.df_chain_energy_grad(vec0, ham, obs, 0.1, 2, norb, nelec,
                                                                       plan=plan))
    assert c == c_ref and all(np.array_equal(cg[x], cg_ref[x]) for x in ("h", "J", "U"))
    # a chain with many terms grows the result block: its allocation fails once, then goes through
    big = synth.df_hamiltonian(r, norb, 210)
    c_big_ref, _ = ffx.df_chain_energy_grad(vec0, big, obs, 0.1, 1, norb, nelec, plan=ref_plan)
    k3, (c_big, _) = _until_success(ffx, lambda: ffx.df_chain_energy_grad(vec0, big, obs, 0.1, 1, norb, nelec,
                                                                          plan=plan))
    assert k3 > 1 and c_big == c_big_ref
    print(f"fault injection: gradients went through at k = {k1}, {k2}, {k3}", flush=True)


def test_batched_call_after_failed_allocations(ffx):
    w = synth.workload_batched(8, seed=2, n_reps=1)
    sectors = [(x.norb, x.nelec) for x in w]
    args = ([x.data["params"] for x in w], [x.data["ham"] for x in w], 1)
    ref = ffx.Batch(sectors, dtype=torch.complex64)
    e_ref, g_ref = ref.lucj_energy_grad(*args)
    print("fault injection: batched call", flush=True)
    # batch creation makes hundreds of allocations (plans, replicated class tables): a sample of them fails
    b = _sampled(ffx, lambda: ffx.Batch(sectors, dtype=torch.complex64), [1, 2, 3, 5, 9, 17, 40, 90, 200, 450])
    b.workspace()
    k, (e, g) = _until_success(ffx, lambda: b.lucj_energy_grad(*args))
    assert k > 1
    np.testing.assert_array_equal(e, e_ref)
    for a, c in zip(g, g_ref):
        np.testing.assert_array_equal(a, c)
    e2, _ = b.lucj_energy_grad(*args)
    np.testing.assert_array_equal(e2, e_ref)
