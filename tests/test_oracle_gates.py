"""Pins for oracle/gates.py against brute-force Fock-space exponentials, closed forms and invariants."""
import numpy as np
import pytest
import scipy.linalg

from oracle import gates as g
from oracle import strings as st
from paper_2605_03123_amd import synth
from jw import Fock

SECTORS = [(3, (1, 2)), (3, (2, 2)), (4, (2, 2)), (4, (3, 1)), (4, (0, 2)), (4, (4, 3))]


def _dims(norb, nelec):
    return st.dim(norb, nelec[0]), st.dim(norb, nelec[1])


@pytest.mark.parametrize("norb,nelec", SECTORS)
def test_orbital_rotation_equals_exponential_of_generator(norb, nelec):
    r = synth.rng(1)
    F = Fock(norb)
    da, db = _dims(norb, nelec)
    vec = synth.random_state(r, da, db)
    Ua = synth.random_unitary(r, norb)
    Ub = synth.random_unitary(r, norb)
    ref = F.restrict(F.orbital_rotation(Ua, Ub), nelec) @ vec.reshape(-1)
    out = g.apply_orbital_rotation(vec, Ua, norb, nelec, U_b=Ub)
    np.testing.assert_allclose(out.reshape(-1), ref, atol=1e-12)


def test_orbital_rotation_special_cases():
    r = synth.rng(2)
    norb = 5
    U = synth.random_unitary(r, norb)
    # one electron per spin: Gamma' = U Gamma U^T  (plain matrix products; pins the transpose)
    vec = synth.random_state(r, 5, 5)
    np.testing.assert_allclose(g.apply_orbital_rotation(vec, U, norb, (1, 1)), U @ vec @ U.T, atol=1e-13)
    # full shell: det(U) per spin; empty shell: identity
    vec = synth.random_state(r, 1, 5)
    np.testing.assert_allclose(g.apply_orbital_rotation(vec, U, norb, (5, 1)),
                               np.linalg.det(U) * vec @ U.T, atol=1e-13)
    vec = synth.random_state(r, 1, 1)
    np.testing.assert_allclose(g.apply_orbital_rotation(vec, U, norb, (0, 0)), vec, atol=0)


def test_orbital_rotation_homomorphism_and_adjoint():
    r = synth.rng(3)
    norb, nelec = 6, (3, 2)
    da, db = _dims(norb, nelec)
    vec = synth.random_state(r, da, db)
    U, V = synth.random_unitary(r, norb), synth.random_unitary(r, norb)
    uv = g.apply_orbital_rotation(vec, U @ V, norb, nelec)
    u_v = g.apply_orbital_rotation(g.apply_orbital_rotation(vec, V, norb, nelec), U, norb, nelec)
    np.testing.assert_allclose(uv, u_v, atol=1e-13)
    back = g.apply_orbital_rotation(g.apply_orbital_rotation(vec, U, norb, nelec), U.conj().T, norb, nelec)
    np.testing.assert_allclose(back, vec, atol=1e-13)
    assert abs(np.linalg.norm(g.apply_orbital_rotation(vec, U, norb, nelec)) - 1) < 1e-13


def test_compound_matrix_rows_and_workers():
    """Selected rows of C_n(U) equal those rows of the whole matrix, in the order asked, for a real and a
    complex U, with the rows spread over worker processes or not; C_1(U) = U."""
    r = synth.rng(11)
    norb, n = 7, 3
    for U in (synth.random_unitary(r, norb), synth.random_unitary(r, norb).real.copy()):
        full = g.compound_matrix(U, n)
        np.testing.assert_allclose(g.compound_matrix(U, 1), U, atol=1e-15)
        rows = np.array([34, 0, 5, 17, 5])
        np.testing.assert_allclose(g.compound_matrix(U, n, rows=rows), full[rows], atol=0)
        g.set_workers(3)
        try:
            np.testing.assert_allclose(g.compound_matrix(U, n, chunk=1), full, atol=1e-15)
            np.testing.assert_allclose(g.compound_matrix(U, n, chunk=1, rows=np.arange(20)), full[:20], atol=1e-15)
        finally:
            g.set_workers(1)


def test_slater_determinant_amplitudes():
    """script-U(U)|HF> has amplitudes det U[J_a, occ] det U[J_b, occ] (Sec. 2.4)."""
    r = synth.rng(4)
    norb, nelec = 6, (2, 3)
    U = synth.random_unitary(r, norb)
    da, db = _dims(norb, nelec)
    hf = synth.hartree_fock(da, db)
    out = g.apply_orbital_rotation(hf, U, norb, nelec)
    occ_a, occ_b = st.occupied_lists(norb, 2), st.occupied_lists(norb, 3)
    a = np.array([np.linalg.det(U[np.ix_(J, [0, 1])]) for J in occ_a])
    b = np.array([np.linalg.det(U[np.ix_(J, [0, 1, 2])]) for J in occ_b])
    np.testing.assert_allclose(out, np.outer(a, b), atol=1e-13)


@pytest.mark.parametrize("norb,nelec", SECTORS)
def test_num_op_sum_equals_exponential(norb, nelec):
    r = synth.rng(5)
    F = Fock(norb)
    da, db = _dims(norb, nelec)
    vec = synth.random_state(r, da, db)
    la, lb = r.normal(size=norb), r.normal(size=norb)
    t = 0.7
    ref = F.restrict(scipy.linalg.expm(-1j * t * F.num_op_sum_gen(la, lb)), nelec) @ vec.reshape(-1)
    out = g.apply_num_op_sum_evolution(vec, la, t, norb, nelec, lam_b=lb)
    np.testing.assert_allclose(out.reshape(-1), ref, atol=1e-13)


@pytest.mark.parametrize("norb,nelec", SECTORS)
def test_diag_coulomb_equals_exponential(norb, nelec):
    r = synth.rng(6)
    F = Fock(norb)
    da, db = _dims(norb, nelec)
    vec = synth.random_state(r, da, db)
    Jaa, Jab, Jbb = (synth.random_symmetric(r, norb, 1.0) for _ in range(3))
    t = 0.3
    gen = F.diag_coulomb_gen(Jaa, Jab, Jbb)
    ref = F.restrict(scipy.linalg.expm(-1j * t * gen), nelec) @ vec.reshape(-1)
    out = g.apply_diag_coulomb_evolution(vec, Jaa, t, norb, nelec, J_ab=Jab, J_bb=Jbb)
    np.testing.assert_allclose(out.reshape(-1), ref, atol=1e-13)
    # single matrix fills every block
    ref1 = F.restrict(scipy.linalg.expm(-1j * t * F.diag_coulomb_gen(Jaa, Jaa, Jaa)), nelec) @ vec.reshape(-1)
    np.testing.assert_allclose(g.apply_diag_coulomb_evolution(vec, Jaa, t, norb, nelec).reshape(-1), ref1,
                               atol=1e-13)


def test_gate_redundancies():
    """Table 1 redundancies: number interaction, number-number interaction, quadratic evolution."""
    r = synth.rng(7)
    norb, nelec = 5, (2, 3)
    da, db = _dims(norb, nelec)
    vec = synth.random_state(r, da, db)
    F = Fock(norb)
    theta = 0.41
    # number interaction exp(i theta n_{2 alpha}) == num-op-sum with lam_a = -e_2, t = theta
    la = np.zeros(norb); la[2] = -1.0
    ref = F.restrict(scipy.linalg.expm(1j * theta * F.n(2, 0)), nelec) @ vec.reshape(-1)
    np.testing.assert_allclose(g.apply_num_op_sum_evolution(vec, la, theta, norb, nelec, lam_b=np.zeros(norb))
                               .reshape(-1), ref, atol=1e-13)
    # number-number interaction exp(i theta n_{1a} n_{3b}) == diag Coulomb with J^{ab}_{13} = -theta, t = 1
    Jab = np.zeros((norb, norb)); Jab[1, 3] = -theta
    Z = np.zeros((norb, norb))
    ref = F.restrict(scipy.linalg.expm(1j * theta * F.n(1, 0) @ F.n(3, 1)), nelec) @ vec.reshape(-1)
    out = g.apply_diag_coulomb_evolution(vec, Z, 1.0, norb, nelec, J_ab=Jab, J_bb=Z)
    np.testing.assert_allclose(out.reshape(-1), ref, atol=1e-13)
    # quadratic Hamiltonian evolution == orbital rotation with U = exp(-i M t)
    M = synth.random_hermitian(r, norb, 1.0)
    ref = F.restrict(scipy.linalg.expm(-1j * 0.8 * F.one_body(M)), nelec) @ vec.reshape(-1)
    out = g.apply_orbital_rotation(vec, scipy.linalg.expm(-1j * 0.8 * M), norb, nelec)
    np.testing.assert_allclose(out.reshape(-1), ref, atol=1e-12)
    # num-op-sum == orbital rotation with U = diag(exp(-i lam t))
    lam = r.normal(size=norb)
    np.testing.assert_allclose(g.apply_num_op_sum_evolution(vec, lam, 0.6, norb, nelec),
                               g.apply_orbital_rotation(vec, np.diag(np.exp(-0.6j * lam)), norb, nelec),
                               atol=1e-13)


@pytest.mark.parametrize("p,q", [(0, 1), (1, 2), (0, 3), (3, 1), (2, 0)])
def test_givens_pair_action(p, q):
    """The Givens formula (with the sign reading for non-adjacent orbitals) equals
    exp(theta (e^{i phi} a^dag_p a_q - h.c.)) and equals the orbital rotation by the 2x2 block."""
    norb, nelec = 4, (2, 3)
    r = synth.rng(8)
    F = Fock(norb)
    da, db = _dims(norb, nelec)
    vec = synth.random_state(r, da, db)
    theta, phi = 0.37, 1.1
    c, s = np.cos(theta), np.exp(1j * phi) * np.sin(theta)
    G = np.eye(norb, dtype=complex)
    G[p, p], G[p, q], G[q, p], G[q, q] = c, s, -np.conj(s), c
    for spin in (0, 1):
        out = g.apply_givens(vec, c, s, p, q, norb, nelec, spin)
        Ua = G if spin == 0 else np.eye(norb)
        Ub = G if spin == 1 else np.eye(norb)
        np.testing.assert_allclose(out, g.apply_orbital_rotation(vec, Ua, norb, nelec, U_b=Ub), atol=1e-13)
        m = F.mode
        gen = theta * (np.exp(1j * phi) * F.cre[m(p, spin)] @ F.ann[m(q, spin)]
                       - np.exp(-1j * phi) * F.cre[m(q, spin)] @ F.ann[m(p, spin)])
        ref = F.restrict(scipy.linalg.expm(gen), nelec) @ vec.reshape(-1)
        np.testing.assert_allclose(out.reshape(-1), ref, atol=1e-12)


def test_one_body_action_and_transition_matrix():
    r = synth.rng(9)
    norb, nelec = 4, (2, 1)
    F = Fock(norb)
    da, db = _dims(norb, nelec)
    vec, lam = synth.random_state(r, da, db), synth.random_state(r, da, db)
    M = r.normal(size=(norb, norb)) + 1j * r.normal(size=(norb, norb))
    ref = F.restrict(F.one_body(M), nelec) @ vec.reshape(-1)
    np.testing.assert_allclose(g.apply_one_body(vec, M, norb, nelec).reshape(-1), ref, atol=1e-13)
    T = g.transition_one_body(lam, vec, norb, nelec)
    for p in range(norb):
        for q in range(norb):
            ref = np.vdot(lam.reshape(-1), F.restrict(F.E(p, q), nelec) @ vec.reshape(-1))
            assert abs(T[p, q] - ref) < 1e-13


@pytest.mark.parametrize("norb,nelec", SECTORS)
def test_diag_coulomb_angle_at_equals_generator_diagonal(norb, nelec):
    # the pointwise angle is twice the diagonal of the Fock-space generator
    r = synth.rng(61)
    F = Fock(norb)
    da, db = _dims(norb, nelec)
    Jaa, Jab, Jbb = (synth.random_symmetric(r, norb, 1.0) for _ in range(3))
    gen = np.diag(F.restrict(F.diag_coulomb_gen(Jaa, Jab, Jbb), nelec)).reshape(da, db)
    idx = [(i, j) for i in range(da) for j in range(db)]
    at = g.diag_coulomb_angle_at(norb, nelec, idx, Jaa, Jab, Jbb)
    np.testing.assert_allclose(at, 2 * gen.reshape(-1), atol=1e-13)
    np.testing.assert_allclose(at, g.diag_coulomb_angle(norb, nelec, Jaa, Jab, Jbb).reshape(-1), atol=1e-13)
