"""GPU parity of sampling (Sec. 4.5.4, 6.1) through the C ABI against the oracle, on the same seeded
uniforms.  A sampled index is decided by a floating-point comparison, and the two sides sum in different
orders; so each GPU index must equal the oracle's unless the target lies within 1e-12 (relative) of the
boundary between the two, and at most a handful of samples may take that exception."""
import numpy as np
import pytest
import torch

from oracle import sampling as osm
from oracle import strings as ost
from paper_2605_03123_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ffx():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_2605_03123_amd import ffx as mod
    return mod


def _dims(norb, nelec):
    return ost.dim(norb, nelec[0]), ost.dim(norb, nelec[1])


def _check_state_samples(got, vec_np, u):
    ref = osm.sample_state(vec_np, u)
    bad = np.flatnonzero(got != ref)
    p = np.abs(vec_np.reshape(-1)) ** 2
    cdf = np.cumsum(p)
    for k in bad:
        # both indices valid and the target at the boundary between them
        lo, hi = sorted((int(got[k]), int(ref[k])))
        assert p[got[k]] > 0
        assert abs(u[k] * cdf[-1] - cdf[lo]) <= 1e-12 * cdf[-1], (k, got[k], ref[k])
        assert np.all(p[lo + 1:hi] == 0)
    assert len(bad) <= 2


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
@pytest.mark.parametrize("norb,nelec", [(4, (2, 2)), (9, (5, 3)), (12, (6, 6)), (5, (0, 5)), (13, (4, 7))])
def test_sample_state(ffx, dtype, norb, nelec):
    r = synth.rng([81, norb, *nelec])
    vec = synth.random_state(r, *_dims(norb, nelec))
    if vec.shape[0] > 3:
        vec[1:3] = 0.0  # zero-probability rows
    t = torch.from_numpy(vec).to(dtype).to("cuda:0")
    x = t.cpu().to(torch.complex128).numpy()
    u = r.random(5000)
    got = ffx.sample_state(t, u, norb, nelec)
    _check_state_samples(got, x, u)


def test_sample_state_edge_cases(ffx):
    norb, nelec = 6, (3, 2)
    da, db = _dims(norb, nelec)
    vec = torch.zeros((da, db), dtype=torch.complex128, device="cuda:0")
    vec[7, 11] = 0.5j  # one configuration holds all the probability
    got = ffx.sample_state(vec, np.array([0.0, 0.5, 0.9999999]), norb, nelec)
    np.testing.assert_array_equal(got, [7 * db + 11] * 3)
    assert ffx.sample_state(vec, np.zeros(0), norb, nelec).size == 0
    with pytest.raises(ffx.FFXError):
        ffx.sample_state(vec, np.array([1.0]), norb, nelec)
    with pytest.raises(ffx.FFXError):
        ffx.sample_state(torch.zeros_like(vec), np.array([0.5]), norb, nelec)


def test_sample_state_full_size(ffx):
    """norb = 16, (8, 8) complex128 (2.65 GB), 20000 samples against the oracle's cumulative sum."""
    norb, nelec = 16, (8, 8)
    r = synth.rng(82)
    vec = synth.random_state(r, 12870, 12870)
    t = torch.from_numpy(vec).to("cuda:0")
    u = r.random(20000)
    got = ffx.sample_state(t, u, norb, nelec)
    _check_state_samples(got, vec, u)


@pytest.mark.parametrize("norb,nelec", [(4, (2, 2)), (8, (3, 5)), (12, (6, 5)), (16, (8, 8)), (32, (4, 4)),
                                        (5, (0, 5))])
def test_sample_slater(ffx, norb, nelec):
    r = synth.rng([83, norb, *nelec])
    Ua, Ub = synth.random_unitary(r, norb), synth.random_unitary(r, norb)
    occ_a = sorted(r.permutation(norb)[:nelec[0]].tolist())
    occ_b = r.permutation(norb)[:nelec[1]].tolist()
    M = 300
    ua, ub = r.random((M, nelec[0])), r.random((M, nelec[1]))
    ma, mb = ffx.sample_slater(norb, nelec, ua, ub, U=Ua, U_b=Ub, occ_a=occ_a, occ_b=occ_b)
    ra, rb = osm.sample_slater(norb, nelec, Ua, ua, U_b=Ub, u_b=ub, occ_a=occ_a, occ_b=occ_b)
    for got, ref, n in ((ma, ra, nelec[0]), (mb, rb, nelec[1])):
        assert all(bin(int(m)).count("1") == n for m in got)
        assert np.all(got < (1 << norb))
        assert (got != ref).sum() <= 1


def test_sample_slater_frequencies(ffx):
    """Many samples: the frequencies of the alpha configurations match |det U[I, occ]|^2."""
    norb, nelec = 6, (3, 1)
    r = synth.rng(84)
    U = synth.random_unitary(r, norb)
    occ = [0, 2, 5]
    M = 200000
    ma, _ = ffx.sample_slater(norb, nelec, r.random((M, 3)), r.random((M, 1)), U=U, occ_a=occ)
    strs = ost.strings(norb, 3)
    freq = np.array([(ma == m).sum() for m in strs]) / M
    p = np.array([abs(np.linalg.det(U[np.ix_([q for q in range(norb) if (int(m) >> q) & 1], occ)])) ** 2
                  for m in strs])
    assert abs(freq.sum() - 1.0) < 1e-12
    assert np.all(np.abs(freq - p) <= 4.5 * np.sqrt(p * (1 - p) / M) + 1e-12)
