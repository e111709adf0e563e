"""Pins for the remaining Table 1 gates of the oracle, its Slater-determinant state and its UCJ forward
pass, against exponentials of the gates' generators on the Jordan-Wigner Fock space (tests/jw.py) and
against special cases that reduce to already pinned functions."""
import numpy as np
import pytest
import scipy.linalg

from oracle import gates as g
from oracle import lucj as ol
from oracle import strings as st
from paper_2605_03123_amd import synth
from jw import Fock

SECTORS = [(3, (1, 2)), (4, (2, 2)), (4, (3, 1)), (4, (0, 2))]


def _dims(norb, nelec):
    return st.dim(norb, nelec[0]), st.dim(norb, nelec[1])


def _hop(F, p, q, s):
    return F.cre[F.mode(p, s)] @ F.ann[F.mode(q, s)]


def _apply(F, gen, nelec, vec):
    return F.restrict(scipy.linalg.expm(gen), nelec) @ vec.reshape(-1)


@pytest.mark.parametrize("norb,nelec", SECTORS)
def test_number_interactions(norb, nelec):
    F = Fock(norb)
    r = synth.rng([51, norb, *nelec])
    vec = synth.random_state(r, *_dims(norb, nelec))
    for p, s in [(0, 0), (norb - 1, 1), (1, 1)]:
        ref = _apply(F, 0.7j * F.n(p, s), nelec, vec)
        np.testing.assert_allclose(g.apply_num_interaction(vec, 0.7, p, s, norb, nelec).reshape(-1), ref, atol=1e-12)
    for p, sg, q, tu in [(0, 0, 1, 1), (1, 0, 1, 1), (0, 0, 2, 0), (2, 1, 2, 1), (2, 1, 0, 0)]:
        ref = _apply(F, -1.3j * F.n(p, sg) @ F.n(q, tu), nelec, vec)
        out = g.apply_num_num_interaction(vec, -1.3, p, sg, q, tu, norb, nelec)
        np.testing.assert_allclose(out.reshape(-1), ref, atol=1e-12)


@pytest.mark.parametrize("norb,nelec", SECTORS)
def test_givens_and_tunneling(norb, nelec):
    F = Fock(norb)
    r = synth.rng([52, norb, *nelec])
    vec = synth.random_state(r, *_dims(norb, nelec))
    for p, q, s in [(0, 1, 0), (2, 0, 1), (0, norb - 1, 0), (1, 2, 1)]:
        th = 0.4 + 0.3 * p - 0.2 * q
        gen = th * (_hop(F, p, q, s) - _hop(F, q, p, s))
        np.testing.assert_allclose(g.apply_givens_rotation(vec, th, p, q, s, norb, nelec).reshape(-1),
                                   _apply(F, gen, nelec, vec), atol=1e-12)
        gen = 1j * th * (_hop(F, p, q, s) + _hop(F, q, p, s))
        np.testing.assert_allclose(g.apply_tunneling_interaction(vec, th, p, q, s, norb, nelec).reshape(-1),
                                   _apply(F, gen, nelec, vec), atol=1e-12)


@pytest.mark.parametrize("norb,nelec", SECTORS)
def test_quadratic_hamiltonian_evolution(norb, nelec):
    F = Fock(norb)
    r = synth.rng([53, norb, *nelec])
    vec = synth.random_state(r, *_dims(norb, nelec))
    Ma, Mb = synth.random_hermitian(r, norb, 0.7), synth.random_hermitian(r, norb, 0.7)
    gen = sum(Ma[p, q] * _hop(F, p, q, 0) + Mb[p, q] * _hop(F, p, q, 1) for p in range(norb) for q in range(norb))
    out = g.apply_quad_ham_evolution(vec, Ma, 0.9, norb, nelec, M_b=Mb)
    np.testing.assert_allclose(out.reshape(-1), _apply(F, -0.9j * gen, nelec, vec), atol=1e-12)


@pytest.mark.parametrize("norb,nelec,occ_a,occ_b", [(4, (2, 2), [3, 1], [0, 2]), (4, (3, 1), [0, 2, 3], [3]),
                                                    (3, (1, 2), None, [2, 0])])
def test_slater_determinant(norb, nelec, occ_a, occ_b):
    F = Fock(norb)
    r = synth.rng([54, norb])
    Ua, Ub = synth.random_unitary(r, norb), synth.random_unitary(r, norb)
    oa = list(range(nelec[0])) if occ_a is None else occ_a
    ob = list(range(nelec[1])) if occ_b is None else occ_b
    # the basis configuration with those orbitals occupied, in the sector basis
    amap_a, amap_b = st.address_map(norb, nelec[0]), st.address_map(norb, nelec[1])
    e = np.zeros(_dims(norb, nelec), dtype=complex)
    e[amap_a[sum(1 << o for o in oa)], amap_b[sum(1 << o for o in ob)]] = 1.0
    ref = F.restrict(F.orbital_rotation(Ua, Ub), nelec) @ e.reshape(-1)
    out = g.slater_determinant(norb, nelec, occ_a=occ_a, occ_b=occ_b, U_a=Ua, U_b=Ub)
    np.testing.assert_allclose(out.reshape(-1), ref, atol=1e-12)
    # closed form (Sec. 2.4): product of the minors U[I, occ] per spin
    Ia, Ib = st.occupied_lists(norb, nelec[0]), st.occupied_lists(norb, nelec[1])
    so = sorted(oa), sorted(ob)
    ma = np.array([np.linalg.det(Ua[np.ix_(I, so[0])]) if len(I) else 1.0 for I in Ia])
    mb = np.array([np.linalg.det(Ub[np.ix_(I, so[1])]) if len(I) else 1.0 for I in Ib])
    np.testing.assert_allclose(out, np.outer(ma, mb), atol=1e-12)


def test_ucj_special_cases():
    norb, nelec, R = 5, (3, 2), 2
    r = synth.rng(55)
    # restricted to the LUCJ layout it is the (separately pinned) LUCJ ansatz
    params = synth.lucj_params(r, norb, R, scale=0.3)
    reps = ol.unpack(params, norb, R)
    U = [scipy.linalg.expm(K) for K, _, _ in reps]
    Js = [Jsame for _, Jsame, _ in reps]
    Jo = [Jopp for _, _, Jopp in reps]
    out = g.apply_ucj(norb, nelec, U, Js, J_ab=Jo, J_bb=Js)
    np.testing.assert_allclose(out, ol.apply_lucj(params, norb, nelec, R), atol=1e-12)
    # J = 0: every U_k D_k U_k^dag is the identity, leaving the final rotation on HF
    Ua = [synth.random_unitary(r, norb) for _ in range(R)]
    Ub = [synth.random_unitary(r, norb) for _ in range(R)]
    Fa, Fb = synth.random_unitary(r, norb), synth.random_unitary(r, norb)
    Z = [np.zeros((norb, norb))] * R
    out = g.apply_ucj(norb, nelec, Ua, Z, U_b=Ub, final_a=Fa, final_b=Fb)
    np.testing.assert_allclose(out, g.slater_determinant(norb, nelec, U_a=Fa, U_b=Fb), atol=1e-12)
    # one repetition against the Fock-space product of exponentials, per-spin U and a full J
    norb, nelec = 3, (2, 1)
    F = Fock(norb)
    U1a, U1b = synth.random_unitary(r, norb), synth.random_unitary(r, norb)
    Jaa, Jbb = synth.random_symmetric(r, norb, 0.5), synth.random_symmetric(r, norb, 0.5)
    Jab = r.normal(0, 0.5, (norb, norb))
    rot = F.orbital_rotation(U1a, U1b)
    D = scipy.linalg.expm(-1j * F.diag_coulomb_gen(Jaa, Jab, Jbb))
    hf = np.zeros(_dims(norb, nelec), dtype=complex)
    hf[0, 0] = 1.0
    ref = F.restrict(rot @ D @ rot.conj().T, nelec) @ hf.reshape(-1)
    out = g.apply_ucj(norb, nelec, [U1a], [Jaa], U_b=[U1b], J_ab=[Jab], J_bb=[Jbb])
    np.testing.assert_allclose(out.reshape(-1), ref, atol=1e-12)


@pytest.mark.parametrize("norb,nelec", [(3, (1, 2)), (4, (2, 2))])
def test_diagonal_gates_in_a_rotated_basis(norb, nelec):
    """exp(-i t sum lam_p n~_p) and exp(-1/2 i t sum J n~ n~) with n~_p = script-U(B) n_p script-U(B)^dag."""
    F = Fock(norb)
    r = synth.rng([56, norb, *nelec])
    vec = synth.random_state(r, *_dims(norb, nelec))
    B = synth.random_unitary(r, norb)
    lam = r.normal(0, 1, norb)
    nt = [[F.rotated_number(B, p, s) for p in range(norb)] for s in (0, 1)]
    gen = sum(lam[p] * (nt[0][p] + nt[1][p]) for p in range(norb))
    out = g.apply_in_basis(vec, B, lambda v: g.apply_num_op_sum_evolution(v, lam, 0.6, norb, nelec), norb, nelec)
    np.testing.assert_allclose(out.reshape(-1), _apply(F, -0.6j * gen, nelec, vec), atol=1e-12)
    J = synth.random_symmetric(r, norb, 0.5)
    gen = sum(0.5 * J[p, q] * nt[s][p] @ nt[t][q] for p in range(norb) for q in range(norb)
              for s in (0, 1) for t in (0, 1))
    out = g.apply_in_basis(vec, B, lambda v: g.apply_diag_coulomb_evolution(v, J, 0.6, norb, nelec), norb, nelec)
    np.testing.assert_allclose(out.reshape(-1), _apply(F, -0.6j * gen, nelec, vec), atol=1e-12)
