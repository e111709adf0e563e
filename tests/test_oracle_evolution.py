"""Pins for the Trotter-error path of the oracle (Sec. 6.2): the 2D Hubbard model in
the DF form the library takes, exact evolution, and the Trotter error itself.

* The Hubbard data against the model as the paper writes it, built on the
  Jordan-Wigner Fock space from hopping and n_a n_b operators (tests/jw.py).
* evolve_exact against the spectral decomposition of the explicit sector
  matrix, against the closed form of a one-body Hamiltonian (an orbital
  rotation by expm(-i h t)), and against the Fock-space exponential of the
  Hubbard model.
* trotter_error: orders of the product formulas (error ratio for doubled step
  counts: 2 for S_0, 4 for S_1, 16 for S_2) and its limits (no error when
  the terms commute, the exact value when the time is zero).
"""
import numpy as np
import pytest
import scipy.linalg

from oracle import gates as g
from oracle import hamiltonian as H
from oracle import hamiltonian as oh
from oracle import strings as st
from paper_2605_03123_amd import synth
from jw import Fock


def _dims(norb, nelec):
    return st.dim(norb, nelec[0]), st.dim(norb, nelec[1])


def _hubbard_fock(F, nx, ny, t, U, periodic_x, periodic_y):
    """-t sum_<pq>,s (a+_ps a_qs + a+_qs a_ps) + U sum_p n_pa n_pb on the Fock space,
    neighbours enumerated here independently of synth.lattice_edges."""
    n = nx * ny
    op = np.zeros((F.dim, F.dim))
    for p in range(n):
        x, y = p % nx, p // nx
        nbrs = []
        if x + 1 < nx or (periodic_x and nx > 2):
            nbrs.append(((x + 1) % nx) + nx * y)
        if y + 1 < ny or (periodic_y and ny > 2):
            nbrs.append(x + nx * ((y + 1) % ny))
        for q in nbrs:
            op += -t * (F.E(p, q) + F.E(q, p))
    for p in range(n):
        op += U * F.n(p, 0) @ F.n(p, 1)
    return op


@pytest.mark.parametrize("nx,ny,px,nelec", [(4, 1, True, (1, 1)), (4, 1, True, (2, 1)), (2, 2, False, (1, 1)),
                                            (2, 2, False, (2, 2))])
def test_hubbard_df_form_is_the_hubbard_model(nx, ny, px, nelec):
    norb = nx * ny
    ham = synth.hubbard_2d(nx, ny, t=1.0, U=8.0, periodic_x=px)
    F = Fock(norb)
    Hs = F.restrict(_hubbard_fock(F, nx, ny, 1.0, 8.0, px, False), nelec)
    da, db = _dims(norb, nelec)
    vec = synth.random_state(synth.rng([31, nx, ny]), da, db)
    out = H.apply_df_hamiltonian(vec, ham, norb, nelec)
    np.testing.assert_allclose(out.reshape(-1), Hs @ vec.reshape(-1), atol=1e-12)
    # and the exact evolution of that model
    ex = H.evolve_exact(vec, ham, 0.7, norb, nelec)
    np.testing.assert_allclose(ex.reshape(-1), scipy.linalg.expm(-0.7j * Hs) @ vec.reshape(-1), atol=1e-12)


def test_hubbard_lattice_and_filling():
    # 4 x y, periodic in x: 4 horizontal pairs per row, 4 vertical pairs per row gap
    for y in range(2, 9):
        assert len(synth.lattice_edges(4, y)) == 4 * y + 4 * (y - 1)
        na, nb = synth.hubbard_filling(4, y)
        assert na + nb == y and na - nb in (0, 1)  # 1/8 of 8y spin orbitals
    assert synth.hubbard_filling(4, 8) == (4, 4)
    with pytest.raises(ValueError):
        synth.lattice_edges(2, 3, periodic_x=True)


def _explicit(ham, norb, nelec):
    da, db = _dims(norb, nelec)
    D = da * db
    M = np.zeros((D, D), dtype=complex)
    for k in range(D):
        e = np.zeros(D, dtype=complex)
        e[k] = 1.0
        M[:, k] = H.apply_df_hamiltonian(e.reshape(da, db), ham, norb, nelec).reshape(-1)
    return M


@pytest.mark.parametrize("norb,nelec,L,time", [(5, (2, 2), 2, 1.3), (6, (3, 1), 1, -0.6), (4, (0, 2), 2, 2.0)])
def test_evolve_exact_matches_spectral_decomposition(norb, nelec, L, time):
    r = synth.rng([32, norb, L])
    ham = synth.df_hamiltonian(r, norb, L, h_scale=1.0, j_scale=0.5)
    da, db = _dims(norb, nelec)
    vec = synth.random_state(r, da, db)
    M = _explicit(ham, norb, nelec)
    assert np.abs(M - M.conj().T).max() < 1e-12
    w, W = np.linalg.eigh(M)
    ref = W @ (np.exp(-1j * time * w) * (W.conj().T @ vec.reshape(-1)))
    out = H.evolve_exact(vec, ham, time, norb, nelec)
    np.testing.assert_allclose(out.reshape(-1), ref, atol=1e-12)


def test_evolve_exact_one_body_closed_form():
    norb, nelec = 6, (3, 2)
    r = synth.rng(33)
    h = synth.random_symmetric(r, norb, 1.0)
    ham = synth.DFHamiltonian(h=h, J=np.zeros((0, norb, norb)), U=np.zeros((0, norb, norb), dtype=complex))
    vec = synth.random_state(r, *_dims(norb, nelec))
    ref = g.apply_orbital_rotation(vec, scipy.linalg.expm(-0.9j * h), norb, nelec)
    np.testing.assert_allclose(H.evolve_exact(vec, ham, 0.9, norb, nelec), ref, atol=1e-12)


def test_evolve_exact_reversible_and_norm_preserving():
    nx, ny = 4, 2
    ham = synth.hubbard_2d(nx, ny)
    nelec = synth.hubbard_filling(nx, ny)
    vec = synth.random_state(synth.rng(34), *_dims(8, nelec))
    fwd = H.evolve_exact(vec, ham, 1.0, 8, nelec)
    assert abs(np.linalg.norm(fwd) - 1.0) < 1e-12
    np.testing.assert_allclose(H.evolve_exact(fwd, ham, -1.0, 8, nelec), vec, atol=1e-12)
    # energy is conserved by the exact evolution
    e0 = H.df_energy(vec, ham, 8, nelec).real
    e1 = H.df_energy(fwd, ham, 8, nelec).real
    assert abs(e0 - e1) < 1e-11


@pytest.mark.parametrize("order,ratio", [(0, 2.0), (1, 4.0), (2, 16.0)])
def test_trotter_error_order(order, ratio):
    """Global error of S_k over a fixed time falls as n_steps^-p, p = 1, 2, 4."""
    nx, ny = 4, 2
    ham = synth.hubbard_2d(nx, ny)
    nelec = synth.hubbard_filling(nx, ny)
    vec = synth.random_state(synth.rng(35), *_dims(8, nelec))
    time = 0.5
    exact = H.evolve_exact(vec, ham, time, 8, nelec)
    n = {0: 64, 1: 16, 2: 8}[order]
    e1 = H.trotter_error(vec, ham, time, 8, nelec, n, order, exact=exact)
    e2 = H.trotter_error(vec, ham, time, 8, nelec, 2 * n, order, exact=exact)
    assert e1 > 1e-9
    assert abs(e1 / e2 / ratio - 1.0) < 0.15


def test_trotter_error_limits():
    nx, ny = 4, 2
    nelec = synth.hubbard_filling(nx, ny)
    vec = synth.random_state(synth.rng(36), *_dims(8, nelec))
    # U = 0: a single one-body term, nothing to split
    free = synth.hubbard_2d(nx, ny, U=0.0)
    assert H.trotter_error(vec, free, 1.0, 8, nelec, 1, 0) < 1e-12
    # zero time
    assert H.trotter_error(vec, synth.hubbard_2d(nx, ny), 0.0, 8, nelec, 1, 1) < 1e-14


# ---------------------------------------------------------------------------
# Trotter steps of the diagonal Coulomb Hamiltonian (Eq. diagonal-coulomb-hamiltonian, Sec. 4.5.3)
# ---------------------------------------------------------------------------

def _dc_case(seed, norb=3):
    r = synth.rng(seed)
    h = synth.random_symmetric(r, norb, 1.0)
    Jaa, Jbb = synth.random_symmetric(r, norb, 0.8), synth.random_symmetric(r, norb, 0.8)
    Jab = r.normal(0, 0.8, (norb, norb))  # J^{ba} = J_ab^T, so J_ab need not be symmetric
    return h, Jaa, Jab, Jbb


@pytest.mark.parametrize("order", [0, 1, 2])
def test_diag_coulomb_trotter_single_term_is_exact(order):
    """With one of the two terms zero, every product formula is the exact evolution of the other, which
    the Fock space gives as the exponential of its generator (one-body term, spin-resolved J)."""
    norb, nelec, T = 3, (1, 2), 0.7
    h, Jaa, Jab, Jbb = _dc_case(62)
    F = Fock(norb)
    vec = synth.random_state(synth.rng(63), 3, 3)
    Z = np.zeros((norb, norb))
    for hh, (a, b, c) in ((h, (Z, Z, Z)), (Z, (Jaa, Jab, Jbb))):
        H = F.restrict(F.one_body(hh) + F.diag_coulomb_gen(a, b, c), nelec)
        ref = (scipy.linalg.expm(-1j * T * H) @ vec.reshape(-1)).reshape(vec.shape)
        got = oh.simulate_trotter_diag_coulomb(vec, hh, a, T, norb, nelec, J_ab=b, J_bb=c, n_steps=2, order=order)
        np.testing.assert_allclose(got, ref, atol=1e-13)


@pytest.mark.parametrize("order,ratio", [(0, 2.0), (1, 4.0), (2, 16.0)])
def test_diag_coulomb_trotter_error_order(order, ratio):
    """Against the Fock-space exp(-i T H) of the whole Hamiltonian: doubling the steps divides the error by
    2, 4 and 16 for S_0, S_1 and S_2 (a dropped, misplaced or mis-timed term breaks the order)."""
    norb, nelec, T = 3, (2, 1), 0.5
    h, Jaa, Jab, Jbb = _dc_case(64)
    F = Fock(norb)
    H = F.restrict(F.one_body(h) + F.diag_coulomb_gen(Jaa, Jab, Jbb), nelec)
    vec = synth.random_state(synth.rng(65), 3, 3)
    exact = (scipy.linalg.expm(-1j * T * H) @ vec.reshape(-1)).reshape(vec.shape)
    np.testing.assert_allclose(oh.apply_diag_coulomb_hamiltonian(vec, h, Jaa, norb, nelec, Jab, Jbb).reshape(-1),
                               H @ vec.reshape(-1), atol=1e-13)
    n = 8 if order < 2 else 4
    e1 = np.linalg.norm(oh.simulate_trotter_diag_coulomb(vec, h, Jaa, T, norb, nelec, Jab, Jbb, n, order) - exact)
    e2 = np.linalg.norm(oh.simulate_trotter_diag_coulomb(vec, h, Jaa, T, norb, nelec, Jab, Jbb, 2 * n, order) - exact)
    assert abs(e1 / e2 - ratio) <= 0.15 * ratio, (e1, e2)


@pytest.mark.parametrize("order", [0, 1, 2])
def test_hubbard_as_diag_coulomb_equals_df_form(order):
    """The Hubbard model as printed (J_ab = U I) and its DF form (one identity-basis term J = U I with h shifted
    by -U/2) differ term by term only by phases of the total number operator, which is constant in a sector:
    their product formulas agree, and the diagonal Coulomb form is the model on the Fock space."""
    nx, ny = 4, 1
    norb, nelec = 4, (2, 1)
    h, Jaa, Jab, Jbb = synth.hubbard_2d_diag_coulomb(nx, ny)
    F = Fock(norb)
    hop = F.one_body(h)
    nn = sum(F.n(p, 0) @ F.n(p, 1) for p in range(norb))
    np.testing.assert_allclose(F.one_body(h) + F.diag_coulomb_gen(Jaa, Jab, Jbb), hop + 8.0 * nn, atol=1e-13)
    vec = synth.random_state(synth.rng(66), 6, 4)
    got = oh.simulate_trotter_diag_coulomb(vec, h, Jaa, 0.6, norb, nelec, Jab, Jbb, n_steps=3, order=order)
    ref = oh.simulate_trotter(vec, synth.hubbard_2d(nx, ny, periodic_x=True), 0.6, norb, nelec, n_steps=3,
                              order=order)
    np.testing.assert_allclose(got, ref, atol=1e-13)
