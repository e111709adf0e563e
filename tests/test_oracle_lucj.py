"""Pins for oracle/lucj.py: Fock-space exponentials, J = 0 and U = I closed forms, adjoint vs FD."""
import numpy as np
import pytest
import scipy.linalg

from oracle import lucj
from oracle import strings as st
from paper_2605_03123_amd import synth
from jw import Fock


def test_lucj_matches_fock_space_product():
    norb, nelec, n_reps = 3, (2, 1), 2
    r = synth.rng(21)
    params = synth.lucj_params(r, norb, n_reps, scale=0.3)
    F = Fock(norb)
    B = F.sector_basis(nelec)
    hf = np.zeros(F.dim)
    hf[0b0011 | (0b001 << norb)] = 1.0   # alpha {0,1}, beta {0}
    assert np.allclose(B.T @ hf, synth.hartree_fock(3, 3).reshape(-1))
    v = hf.astype(complex)
    for K, Js, Jo in lucj.unpack(params, norb, n_reps):
        U = scipy.linalg.expm(K)
        D = scipy.linalg.expm(-1j * F.diag_coulomb_gen(Js, Jo, Js))
        v = F.orbital_rotation(U) @ D @ F.orbital_rotation(U.conj().T) @ v
    np.testing.assert_allclose(lucj.apply_lucj(params, norb, nelec, n_reps).reshape(-1), B.T @ v, atol=1e-12)


def test_zero_interaction_gives_hartree_fock():
    norb, nelec, n_reps = 6, (3, 2), 2
    params = synth.lucj_params(synth.rng(22), norb, n_reps)
    per = 2 * norb * norb + 2 * norb - 1
    for k in range(n_reps):
        params[k * per + 2 * norb * norb:(k + 1) * per] = 0.0
    out = lucj.apply_lucj(params, norb, nelec, n_reps)
    np.testing.assert_allclose(out, synth.hartree_fock(20, 15), atol=1e-13)


def test_identity_rotation_gives_phase_on_hartree_fock():
    norb, nelec, n_reps = 6, (3, 3), 3
    params = synth.lucj_params(synth.rng(23), norb, n_reps)
    per = 2 * norb * norb + 2 * norb - 1
    phase = 0.0
    for k in range(n_reps):
        params[k * per:k * per + 2 * norb * norb] = 0.0
        js = params[k * per + 2 * norb * norb:k * per + 2 * norb * norb + norb - 1]
        jo = params[k * per + 2 * norb * norb + norb - 1:(k + 1) * per]
        # HF has orbitals 0,1,2 of each spin occupied: same-spin pairs (0,1),(1,2) twice, on-site 0..2
        phase += 2 * (js[0] + js[1]) + jo[0] + jo[1] + jo[2]
    out = lucj.apply_lucj(params, norb, nelec, n_reps)
    np.testing.assert_allclose(out, np.exp(-1j * phase) * synth.hartree_fock(20, 20), atol=1e-13)


def test_adjoint_gradient_matches_finite_differences():
    norb, nelec, n_reps = 4, (2, 1), 2
    r = synth.rng(24)
    params = synth.lucj_params(r, norb, n_reps, scale=0.3)
    ham = synth.df_hamiltonian(r, norb, 2)
    E, grad = lucj.grad_adjoint(params, ham, norb, nelec, n_reps)
    assert abs(E - lucj.energy(params, ham, norb, nelec, n_reps)) < 1e-13
    fd = lucj.grad_fd(params, ham, norb, nelec, n_reps)
    np.testing.assert_allclose(grad, fd, atol=1e-8)


def test_hermitian_part_of_generator_has_zero_gradient():
    """K = A - A^dag is blind to Hermitian A, so grad . (Hermitian direction) = 0."""
    norb, nelec, n_reps = 4, (2, 2), 1
    r = synth.rng(25)
    params = synth.lucj_params(r, norb, n_reps, scale=0.3)
    ham = synth.df_hamiltonian(r, norb, 2)
    _, grad = lucj.grad_adjoint(params, ham, norb, nelec, n_reps)
    Hm = synth.random_hermitian(r, norb, 1.0)
    d = np.zeros_like(params)
    d[:norb * norb] = Hm.real.reshape(-1)
    d[norb * norb:2 * norb * norb] = Hm.imag.reshape(-1)
    assert abs(grad @ d) < 1e-12
