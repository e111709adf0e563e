"""Pins for oracle/hamiltonian.py: DF action vs explicit rotated number operators, product
formulas vs exponentials, the commuting special case, local-error order, reversibility."""
import numpy as np
import pytest
import scipy.linalg

from oracle import gates as g
from oracle import hamiltonian as H
from oracle import strings as st
from paper_2605_03123_amd import synth
from jw import Fock


def _ham(seed, norb, L, complex_u=False):
    r = synth.rng(seed)
    ham = synth.df_hamiltonian(r, norb, L)
    if complex_u:
        ham.U = np.array([synth.random_unitary(r, norb) for _ in range(L)])
    return ham


@pytest.mark.parametrize("norb,nelec,complex_u", [(3, (1, 2), False), (3, (2, 2), True), (4, (2, 2), False)])
def test_df_action_matches_rotated_number_operators(norb, nelec, complex_u):
    ham = _ham(11, norb, 2, complex_u)
    F = Fock(norb)
    da, db = st.dim(norb, nelec[0]), st.dim(norb, nelec[1])
    vec = synth.random_state(synth.rng(12), da, db)
    Hs = F.restrict(F.df_hamiltonian(ham.h, ham.J, ham.U), nelec)
    ref = Hs @ vec.reshape(-1)
    out = H.apply_df_hamiltonian(vec, ham, norb, nelec)
    np.testing.assert_allclose(out.reshape(-1), ref, atol=1e-12)
    E = H.df_energy(vec, ham, norb, nelec)
    assert abs(E.imag) < 1e-12
    assert abs(E.real - np.vdot(vec.reshape(-1), ref).real) < 1e-12


@pytest.mark.parametrize("order", [0, 1, 2])
def test_trotter_step_matches_product_of_exponentials(order):
    norb, nelec = 3, (2, 1)
    ham = _ham(13, norb, 2)
    F = Fock(norb)
    da, db = st.dim(norb, nelec[0]), st.dim(norb, nelec[1])
    vec = synth.random_state(synth.rng(14), da, db)
    terms = [F.one_body(ham.h).astype(complex)]
    for J, U in zip(ham.J, ham.U):
        t2 = np.zeros((F.dim, F.dim), dtype=complex)
        nr = [[F.rotated_number(U, p, s) for p in range(norb)] for s in (0, 1)]
        for s in (0, 1):
            for t in (0, 1):
                for p in range(norb):
                    for q in range(norb):
                        t2 += 0.5 * J[p, q] * nr[s][p] @ nr[t][q]
        terms.append(t2)
    terms = [F.restrict(T, nelec) for T in terms]

    def S(k, dt):
        if k == 0:
            M = np.eye(da * db, dtype=complex)
            for T in terms:
                M = scipy.linalg.expm(-1j * dt * T) @ M
            return M
        if k == 1:
            M = np.eye(da * db, dtype=complex)
            for T in terms:
                M = scipy.linalg.expm(-0.5j * dt * T) @ M
            for T in reversed(terms):
                M = scipy.linalg.expm(-0.5j * dt * T) @ M
            return M
        u = 1 / (4 - 4 ** (1 / (2 * k - 1)))
        A, B = S(k - 1, u * dt), S(k - 1, (1 - 4 * u) * dt)
        return A @ A @ B @ A @ A

    dt = 0.13
    ref = S(order, dt) @ vec.reshape(-1)
    out = H.trotter_step(vec, ham, dt, norb, nelec, order)
    np.testing.assert_allclose(out.reshape(-1), ref, atol=1e-12)


def test_commuting_case_is_exact():
    """U_t = I and diagonal h: every term is diagonal, so S_0 equals exp(-i H T)."""
    norb, nelec = 5, (2, 3)
    r = synth.rng(15)
    ham = synth.df_hamiltonian(r, norb, 3)
    ham.h = np.diag(np.diag(ham.h))
    ham.U = np.array([np.eye(norb, dtype=complex)] * 3)
    da, db = st.dim(norb, nelec[0]), st.dim(norb, nelec[1])
    vec = synth.random_state(r, da, db)
    out = H.simulate_trotter(vec, ham, 0.9, norb, nelec, n_steps=3, order=0)
    # closed form: phase exp(-i T (sum eps_p N_p + sum_t 1/2 N^T J_t N))
    xa, xb = st.occupations(norb, nelec[0]), st.occupations(norb, nelec[1])
    eps = np.diag(ham.h)
    ang = (xa @ eps)[:, None] + (xb @ eps)[None, :]
    for J in ham.J:
        Nsum = xa[:, None, :] + xb[None, :, :]
        ang = ang + 0.5 * np.einsum("abp,pq,abq->ab", Nsum, J, Nsum)
    np.testing.assert_allclose(out, np.exp(-0.9j * ang) * vec, atol=1e-12)


def _sector_H(ham, norb, nelec):
    da, db = st.dim(norb, nelec[0]), st.dim(norb, nelec[1])
    cols = []
    for k in range(da * db):
        e = np.zeros(da * db, dtype=complex)
        e[k] = 1
        cols.append(H.apply_df_hamiltonian(e.reshape(da, db), ham, norb, nelec).reshape(-1))
    return np.array(cols).T


@pytest.mark.parametrize("order,slope", [(0, 2), (1, 3), (2, 5)])
def test_local_error_order(order, slope):
    """||S_k(dt) psi - exp(-i H dt) psi|| scales as dt^(2k+1) for k >= 1 and dt^2 for k = 0."""
    norb, nelec = 4, (2, 2)
    ham = _ham(16, norb, 3)
    Hm = _sector_H(ham, norb, nelec)
    vec = synth.random_state(synth.rng(17), 6, 6)
    dts = [0.04, 0.02] if order < 2 else [0.2, 0.1]
    errs = []
    for dt in dts:
        exact = scipy.linalg.expm(-1j * dt * Hm) @ vec.reshape(-1)
        errs.append(np.linalg.norm(H.trotter_step(vec, ham, dt, norb, nelec, order).reshape(-1) - exact))
    measured = np.log(errs[0] / errs[1]) / np.log(2)
    assert abs(measured - slope) < 0.25, (errs, measured)


def test_reversibility():
    norb, nelec = 6, (3, 3)
    ham = _ham(18, norb, 3)
    vec = synth.random_state(synth.rng(19), 20, 20)
    fwd = H.trotter_step(vec, ham, 0.1, norb, nelec, 0)
    # inverse of S_0(dt): terms in reverse order with -dt
    back = fwd
    for t in reversed(range(ham.n_terms)):
        back = H.evolve_two_body(back, ham.J[t], ham.U[t], -0.1, norb, nelec)
    back = H.evolve_one_body(back, ham.h, -0.1, norb, nelec)
    np.testing.assert_allclose(back, vec, atol=1e-13)


def test_slater_energy_by_wick():
    """Energy of a Slater determinant from its one-body density (Wick's theorem) equals the oracle."""
    norb, nelec = 6, (3, 2)
    r = synth.rng(20)
    ham = synth.df_hamiltonian(r, norb, 3)
    ham.U = np.array([synth.random_unitary(r, norb) for _ in range(3)])
    W = synth.random_unitary(r, norb)
    vec = g.apply_orbital_rotation(synth.hartree_fock(20, 15), W, norb, nelec)
    # D^sigma_pq = <a^dag_p a_q> = sum_{k occ} W_pk conj(W_qk)... as <a^dag_p a_q> = (W P W^dag)_qp
    D = []
    for n in nelec:
        P = np.diag([1.0] * n + [0.0] * (norb - n))
        D.append((W @ P @ W.conj().T).T)
    E = sum(np.sum(ham.h * Ds) for Ds in D)
    for J, U in zip(ham.J, ham.U):
        # density in the rotated basis: <n^(t)_p n^(t)_q>; Dr = U^dag-rotated densities
        Dr = [U.T @ Ds @ U.conj() for Ds in D]   # <b^dag_p b_q> with b^dag_p = sum_i U_ip a^dag_i
        occ = [np.real(np.diag(x)) for x in Dr]
        for s in (0, 1):
            for t in (0, 1):
                for p in range(norb):
                    for q in range(norb):
                        val = occ[s][p] * occ[t][q]
                        if s == t:
                            val += (p == q) * occ[s][p] - Dr[s][p, q] * Dr[s][q, p]
                        E += 0.5 * J[p, q] * val
    Eo = H.df_energy(vec, ham, norb, nelec)
    assert abs(Eo.real - np.real(E)) < 1e-12
    assert abs(Eo.imag) < 1e-12


def _jw_chain_energy(F, vec0, ham, obs, dt, n_steps, nelec):
    """The same chain with Fock-space exponentials (independent of the oracle)."""
    B = F.sector_basis(nelec)
    psi = B @ vec0.reshape(-1)
    for _ in range(n_steps):
        psi = F.orbital_rotation(scipy.linalg.expm(-1j * dt * np.asarray(ham.h))) @ psi
        for t in range(ham.J.shape[0]):
            U = np.asarray(ham.U[t])
            G = F.diag_coulomb_gen(ham.J[t], ham.J[t], ham.J[t])
            R = F.orbital_rotation(U)
            psi = R @ scipy.linalg.expm(-1j * dt * G) @ R.conj().T @ psi
    H = F.df_hamiltonian(obs.h, obs.J, obs.U)
    return float(np.real(np.vdot(psi, H @ psi)))


def test_df_chain_energy_and_fd_gradient_match_fock_space():
    # N = 3, (1, 2): chain energy and every finite-difference component against Fock space
    norb, nelec, dt, r = 3, (1, 2), 0.15, 2
    rng = synth.rng(70)
    ham = synth.df_hamiltonian(rng, norb, 2)
    obs = synth.df_hamiltonian(rng, norb, 2)
    vec0 = synth.random_state(rng, 3, 3)
    F = Fock(norb)
    e = H.df_chain_energy(vec0, ham, obs, dt, r, norb, nelec)
    assert abs(e - _jw_chain_energy(F, vec0, ham, obs, dt, r, nelec)) < 1e-12
    g = H.df_chain_grad_fd(vec0, ham, obs, dt, r, norb, nelec)
    step = 1e-5
    # spot components of each kind, recomputed in Fock space
    M = np.zeros((norb, norb))
    M[0, 2] = M[2, 0] = 1.0
    ref = (_jw_chain_energy(F, vec0, type(ham)(h=ham.h + step * M, J=ham.J, U=ham.U), obs, dt, r, nelec)
           - _jw_chain_energy(F, vec0, type(ham)(h=ham.h - step * M, J=ham.J, U=ham.U), obs, dt, r, nelec)) / (2 * step)
    assert abs(g["h"][0, 2] - ref) < 1e-8
    Jp, Jm = ham.J.copy(), ham.J.copy()
    Jp[1] += step * M
    Jm[1] -= step * M
    ref = (_jw_chain_energy(F, vec0, type(ham)(h=ham.h, J=Jp, U=ham.U), obs, dt, r, nelec)
           - _jw_chain_energy(F, vec0, type(ham)(h=ham.h, J=Jm, U=ham.U), obs, dt, r, nelec)) / (2 * step)
    assert abs(g["J"][1, 0, 2] - ref) < 1e-8
    A = np.zeros((norb, norb), dtype=complex)
    A[1, 2] = 1j * step
    K = A - A.conj().T
    Up, Um = ham.U.copy(), ham.U.copy()
    Up[0] = Up[0] @ scipy.linalg.expm(K)
    Um[0] = Um[0] @ scipy.linalg.expm(-K)
    ref = (_jw_chain_energy(F, vec0, type(ham)(h=ham.h, J=ham.J, U=Up), obs, dt, r, nelec)
           - _jw_chain_energy(F, vec0, type(ham)(h=ham.h, J=ham.J, U=Um), obs, dt, r, nelec)) / (2 * step)
    assert abs(g["U"][0, 1, 1, 2] - ref) < 1e-8
    # the generator gradient has no component along the Hermitian part of A: d/dRe A_pq = -d/dRe A_qp
    assert np.allclose(g["U"][:, 0], -np.transpose(g["U"][:, 0], (0, 2, 1)), atol=1e-7)
