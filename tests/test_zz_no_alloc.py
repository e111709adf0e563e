"""The allocation-free state sampler (ffx_sample_state_noalloc) against the allocating one
(ffx_sample_state), through the C ABI: the same kernels on the same state and uniforms, so the sampled
addresses must be identical.  Two calls in a row, the second on a smaller state and with fewer samples,
share the library's static scratch array; invalid uniforms and states give -1 on the device, and states
above the scratch limit are refused before any launch."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2605_03123_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ffx():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_2605_03123_amd import ffx as mod
    return mod


def _case(ffx, norb, nelec, dtype, n_samples, seed):
    r = synth.rng([97, seed])
    da, db = synth.dim(norb, nelec[0]), synth.dim(norb, nelec[1])
    vec = synth.random_state(r, da, db)
    vec[2:5] = 0.0  # zero-probability rows
    t = torch.from_numpy(vec).to(dtype).to("cuda:0")
    u = r.random(n_samples)
    ref = ffx.sample_state(t, u, norb, nelec)
    ud = torch.from_numpy(u).to("cuda:0")
    out = torch.full((n_samples,), -7, dtype=torch.int64, device="cuda:0")
    print(f"noalloc sampling norb={norb} nelec={nelec} dtype={dtype} n={n_samples}", flush=True)
    ffx.sample_state_noalloc(t, ud, out, norb, nelec)
    torch.cuda.synchronize()
    return ref, out.cpu().numpy()


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_noalloc_matches_allocating_entry_point(ffx, dtype):
    ref1, got1 = _case(ffx, 12, (6, 6), dtype, 6000, 1)
    np.testing.assert_array_equal(got1, ref1)
    # a second call with a smaller state and fewer samples reuses the scratch array
    ref2, got2 = _case(ffx, 9, (5, 3), dtype, 2500, 2)
    np.testing.assert_array_equal(got2, ref2)


def test_noalloc_invalid_inputs_marked_on_device(ffx):
    norb, nelec = 8, (4, 4)
    vec = torch.zeros((70, 70), dtype=torch.complex128, device="cuda:0")
    u = torch.tensor([0.25, 0.75], dtype=torch.float64, device="cuda:0")
    out = torch.zeros(2, dtype=torch.int64, device="cuda:0")
    ffx.sample_state_noalloc(vec, u, out, norb, nelec)  # zero norm
    assert out.cpu().tolist() == [-1, -1]
    vec[3, 5] = 1.0
    u = torch.tensor([0.5, 1.5, -0.1, 0.0], dtype=torch.float64, device="cuda:0")
    out = torch.zeros(4, dtype=torch.int64, device="cuda:0")
    ffx.sample_state_noalloc(vec, u, out, norb, nelec)
    assert out.cpu().tolist() == [3 * 70 + 5, -1, -1, 3 * 70 + 5]


def test_noalloc_refuses_states_above_the_limit(ffx):
    # 17 orbitals, (8, 9): 24310^2 = 5.9e8 amplitudes > 2^28; refused before any launch
    plan = ffx.get_plan(17, (8, 9), torch.complex64, 0)
    dummy = torch.zeros(4, dtype=torch.float64, device="cuda:0")
    p = ctypes.c_void_p(dummy.data_ptr())
    code = ffx._sstate_na(plan.handle, p, p, 1, p, ffx._stream(dummy.device))
    assert code == -5
    assert "exceeds" in ffx._last_error().decode()
