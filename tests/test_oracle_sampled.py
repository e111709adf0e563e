"""Pin for oracle/sampled.py: single amplitudes equal entries of the full compound-matrix rotation."""
import numpy as np

from oracle import gates as g
from oracle import sampled
from paper_2605_03123_amd import synth


def test_sampled_amplitudes_equal_full_rotation():
    r = synth.rng(31)
    norb, nelec = 7, (3, 4)
    vec = synth.random_state(r, 35, 35)
    Ua, Ub = synth.random_unitary(r, norb), synth.random_unitary(r, norb)
    full = g.apply_orbital_rotation(vec, Ua, norb, nelec, U_b=Ub)
    idx = [(0, 0), (3, 17), (34, 34), (20, 5)]
    out = sampled.rotated_amplitudes(vec, Ua, norb, nelec, idx, U_b=Ub)
    np.testing.assert_allclose(out, [full[i, j] for i, j in idx], atol=1e-14)


def test_blocked_amplitudes_equal_full_rotation():
    # row blocks smaller than the state, a complex64 state, and repeated columns
    r = synth.rng(32)
    norb, nelec = 8, (3, 4)
    vec = synth.random_state(r, 56, 70).astype(np.complex64)
    Ua, Ub = synth.random_unitary(r, norb), synth.random_unitary(r, norb)
    full = g.apply_orbital_rotation(vec.astype(np.complex128), Ua, norb, nelec, U_b=Ub)
    idx = [(0, 0), (3, 17), (55, 69), (20, 5), (41, 17)]
    out = sampled.rotated_amplitudes_blocked(vec, Ua, norb, nelec, idx, U_b=Ub, block=9)
    np.testing.assert_allclose(out, [full[i, j] for i, j in idx], atol=1e-14)


def test_diag_coulomb_ham_amplitudes_equal_full_action():
    """Single amplitudes of H psi for diagonal Coulomb Hamiltonians (two-body terms in the identity basis):
    the 4 x 3 Hubbard model and a random one with two dense J, against the full DF action."""
    from oracle import hamiltonian as oh
    from oracle import strings as st
    r = synth.rng(33)
    cases = [(synth.hubbard_2d(4, 3), 12, synth.hubbard_filling(4, 3))]
    norb = 6
    eye = np.eye(norb, dtype=np.complex128)
    cases.append((synth.DFHamiltonian(h=synth.random_symmetric(r, norb, 1.0),
                                      J=np.array([synth.random_symmetric(r, norb, 0.5) for _ in range(2)]),
                                      U=np.array([eye, eye])), norb, (3, 2)))
    for ham, n, ne in cases:
        vec = synth.random_state(r, st.dim(n, ne[0]), st.dim(n, ne[1]))
        full = oh.apply_df_hamiltonian(vec, ham, n, ne)
        idx = [(0, 0), (vec.shape[0] - 1, vec.shape[1] - 1), (vec.shape[0] // 2, 1)]
        out = sampled.diag_coulomb_ham_amplitudes(ham, n, ne, idx, lambda i: vec[i, :], lambda j: vec[:, j])
        np.testing.assert_allclose(out, [full[i, j] for i, j in idx], atol=1e-13)
