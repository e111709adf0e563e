"""The dense (compound-matrix) form of an orbital rotation on the FP64 matrix cores, through the C ABI:
against the oracle's compound-matrix rotation (<= 1e-12, complex128), against the Givens path at 14
orbitals, and its argument checks."""
import numpy as np
import pytest
import torch

from oracle import gates as og
from oracle import strings as ost
from paper_2605_03123_amd import synth
from errlog import record

pytestmark = pytest.mark.gpu

CASES = [(1, (0, 1)), (2, (1, 1)), (3, (3, 1)), (4, (2, 2)), (5, (2, 3)), (7, (3, 4)), (8, (4, 4)), (8, (1, 7)),
         (9, (4, 5)), (10, (5, 5)), (11, (5, 4)), (12, (6, 6)), (12, (8, 3))]


@pytest.fixture(scope="module")
def ffx():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_2605_03123_amd import ffx as mod
    return mod


def _host(t):
    return t.detach().cpu().to(torch.complex128).numpy()


@pytest.mark.parametrize("norb,nelec", CASES)
def test_dense_rotation_matches_oracle(ffx, norb, nelec):
    r = synth.rng([71, norb, *nelec])
    da, db = ost.dim(norb, nelec[0]), ost.dim(norb, nelec[1])
    vec = torch.from_numpy(synth.random_state(r, da, db)).to("cuda:0")
    x = _host(vec)
    Ua, Ub = synth.random_unitary(r, norb), synth.random_unitary(r, norb)
    print(f"dense rotation norb={norb} nelec={nelec}", flush=True)
    out = ffx.apply_orbital_rotation_dense(vec, Ua, norb, nelec, U_b=Ub)
    err = float(np.max(np.abs(_host(out) - og.apply_orbital_rotation(x, Ua, norb, nelec, U_b=Ub))))
    assert record("dense_rotation", torch.complex128, "amplitude", err, 1e-12, norb=norb) <= 1e-12
    out = ffx.apply_orbital_rotation_dense(vec, Ua, norb, nelec)
    err = float(np.max(np.abs(_host(out) - og.apply_orbital_rotation(x, Ua, norb, nelec))))
    assert err <= 1e-12
    assert np.array_equal(_host(vec), x)  # functional form


def test_dense_rotation_matches_givens_path_n14(ffx):
    norb, nelec = 14, (7, 7)
    d = ost.dim(norb, 7)
    r = synth.rng(72)
    vec = torch.from_numpy(synth.random_state(r, d, d)).to("cuda:0")
    U = synth.random_unitary(r, norb)
    a = ffx.apply_orbital_rotation_dense(vec, U, norb, nelec)
    b = ffx.apply_orbital_rotation(vec, U, norb, nelec)
    err = torch.max(torch.abs(a - b)).item()
    assert record("dense_vs_givens_n14", torch.complex128, "amplitude", err, 1e-12) <= 1e-12


def test_dense_rotation_arguments(ffx):
    vec64 = torch.zeros((6, 6), dtype=torch.complex64, device="cuda:0")
    with pytest.raises(ffx.FFXError):  # complex128 only
        ffx.apply_orbital_rotation_dense(vec64, np.eye(4), 4, (2, 2))
    vec = torch.zeros((6, 6), dtype=torch.complex128, device="cuda:0")
    with pytest.raises(ffx.FFXError):  # not unitary
        ffx.apply_orbital_rotation_dense(vec, 2 * np.eye(4), 4, (2, 2))
    plan = ffx.get_plan(18, (9, 9), torch.complex128, 0)
    with pytest.raises(ffx.FFXError):  # above 8 electrons and 4096 configurations
        ffx._check(ffx._rot_dense(plan.handle, ffx._vp(vec.data_ptr()), ffx._dptr(ffx._cplx(np.eye(18))), None,
                                  ffx._vp(vec.data_ptr()), ffx._stream(vec.device)))


def test_small_sectors_choose_dense_and_givens_stays_available(ffx, monkeypatch):
    """A standalone rotation of a complex128 sector with at most 128 configurations per spin takes the dense
    form; with FFX_DENSE=0 the plan keeps the Givens sweeps.  Both against the oracle."""
    norb, nelec = 8, (4, 4)
    r = synth.rng(74)
    vec = torch.from_numpy(synth.random_state(r, 70, 70)).to("cuda:0")
    x = _host(vec)
    U = synth.random_unitary(r, norb)
    ref = og.apply_orbital_rotation(x, U, norb, nelec)
    monkeypatch.setenv("FFX_DENSE", "0")
    givens_plan = ffx.Plan(norb, nelec, torch.complex128)
    monkeypatch.delenv("FFX_DENSE")
    dense_plan = ffx.Plan(norb, nelec, torch.complex128)
    for plan in (givens_plan, dense_plan):
        out = ffx.apply_orbital_rotation(vec, U, norb, nelec, plan=plan)
        assert float(np.max(np.abs(_host(out) - ref))) <= 1e-12
    a = ffx.apply_orbital_rotation(vec, U, norb, nelec, plan=givens_plan)
    b = ffx.apply_orbital_rotation_dense(vec, U, norb, nelec, plan=givens_plan)
    c = ffx.apply_orbital_rotation(vec, U, norb, nelec, plan=dense_plan)
    assert torch.equal(b, c)          # the same kernels
    assert not torch.equal(a, c)      # a different summation order
