"""Pins for oracle/sampling.py: a stratified grid of uniforms reproduces every probability of the state
to within one sample; the chain-rule weights of the Slater sampler multiply out, over all orders, to
|det U[I, occ]|^2; empirical frequencies match the determinants."""
from itertools import combinations, permutations

import numpy as np
import pytest

from oracle import gates as g
from oracle import sampling as smp
from oracle import strings as st
from paper_2605_03123_amd import synth


def test_state_sampling_stratified_counts():
    r = synth.rng(71)
    vec = synth.random_state(r, 10, 6)
    vec[3, :] = 0.0  # zero-probability configurations are never drawn
    vec /= np.linalg.norm(vec)
    M = 200000
    u = (np.arange(M) + 0.5) / M
    idx = smp.sample_state(vec, u)
    counts = np.bincount(idx, minlength=vec.size)
    p = np.abs(vec.reshape(-1)) ** 2
    assert np.all(np.abs(counts - M * p) <= 1.0 + 1e-9)
    assert counts.reshape(10, 6)[3].sum() == 0
    # an unnormalised state samples the same distribution
    np.testing.assert_array_equal(smp.sample_state(3.0 * vec, u), idx)


def test_state_sampling_single_configuration():
    vec = np.zeros((4, 4), dtype=complex)
    vec[2, 1] = 1j
    np.testing.assert_array_equal(smp.sample_state(vec, np.array([0.0, 0.3, 0.999999])), [9, 9, 9])


@pytest.mark.parametrize("norb,n", [(4, 2), (5, 3), (5, 1), (6, 2)])
def test_chain_rule_gives_determinants(norb, n):
    r = synth.rng([72, norb, n])
    U = synth.random_unitary(r, norb)
    occ = sorted(r.permutation(norb)[:n].tolist())
    K = smp.slater_kernel(U, occ)
    for S in combinations(range(norb), n):
        total = 0.0
        for order in permutations(S):
            pr, chosen = 1.0, []
            for j in order:
                w = smp.conditional_weights(K, chosen)
                pr *= w[j] / w.sum()
                chosen.append(j)
            total += pr
        ref = abs(np.linalg.det(U[np.ix_(list(S), occ)])) ** 2
        assert abs(total - ref) < 1e-12


def test_slater_sampling_frequencies():
    norb, nelec = 5, (2, 1)
    r = synth.rng(73)
    U = synth.random_unitary(r, norb)
    M = 40000
    ua, ub = r.random((M, 2)), r.random((M, 1))
    ma, mb = smp.sample_slater(norb, nelec, U, ua, u_b=ub, occ_a=[3, 1], occ_b=[4])
    vec = g.slater_determinant(norb, nelec, occ_a=[3, 1], occ_b=[4], U_a=U)
    sa, sb = st.strings(norb, 2), st.strings(norb, 1)
    pa = (np.abs(vec) ** 2).sum(axis=1)
    pb = (np.abs(vec) ** 2).sum(axis=0)
    for masks, strs, p in ((ma, sa, pa), (mb, sb, pb)):
        freq = np.array([(masks == m).sum() for m in strs]) / M
        assert abs(freq.sum() - 1.0) < 1e-12  # every sample is a valid configuration
        assert np.all(np.abs(freq - p) <= 4.5 * np.sqrt(p * (1 - p) / M) + 1e-12)
