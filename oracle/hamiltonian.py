"""Double-factorized Hamiltonian: action, energy, and Trotter-Suzuki product formulas.

H = sum_{pq,sigma} h_pq a^dag_{p sigma} a_{q sigma}
    + 1/2 sum_t sum_{pq,sigma tau} J^(t)_pq n^(t)_{p sigma} n^(t)_{q tau}
(Eq. double-factorized-hamiltonian), with the rotated number operators
n^(t)_{p sigma} = sum_ij U^(t)_ip a^dag_{i sigma} a_{j sigma} U^(t)*_jp.

Since script-U(U) n_p script-U(U)^dag = n^(t)_p when U = U^(t) (Sec. 2.3), each
two-body term equals script-U(U_t) D_t script-U(U_t)^dag with D_t the diagonal
1/2 sum_pq J_pq N_p N_q, N_p = n_{p alpha} + n_{p beta}.

Readings: the one-body term is H_1, applied first in a product formula, then
the two-body terms in array order (Sec. 4.5.3 does not say which term is H_1);
there is no constant term.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg
import scipy.sparse.linalg as spla

from . import gates as g


def two_body_diagonal(J: np.ndarray, norb: int, nelec) -> np.ndarray:
    """D(I_a, I_b) = 1/2 sum_{(p,q) in S} J_pq: the diagonal of 1/2 sum J_pq N_p N_q."""
    return 0.5 * g.diag_coulomb_angle(norb, nelec, J)


def apply_df_hamiltonian(vec: np.ndarray, ham, norb: int, nelec) -> np.ndarray:
    """H psi for the double-factorized Hamiltonian."""
    out = g.apply_one_body(vec, ham.h, norb, nelec)
    for t in range(ham.n_terms):
        U = ham.U[t]
        phi = g.apply_orbital_rotation(vec, U.conj().T, norb, nelec)
        phi = two_body_diagonal(ham.J[t], norb, nelec) * phi
        out = out + g.apply_orbital_rotation(phi, U, norb, nelec)
    return out


def df_energy(vec: np.ndarray, ham, norb: int, nelec) -> complex:
    """<psi|H|psi> (the paper's np.vdot(vec, linop @ vec), Sec. 4.2).  Real part is the energy."""
    return np.vdot(vec, apply_df_hamiltonian(vec, ham, norb, nelec))


def evolve_exact(vec: np.ndarray, ham, time: float, norb: int, nelec) -> np.ndarray:
    """exp(-i H time) psi: the exact evolution that Trotter errors are measured
    against (Sec. 6.2).  H acts through apply_df_hamiltonian above; scipy's
    expm_multiply (a library step) takes the exponential of that operator."""
    shape = vec.shape
    n = vec.size

    def mv(x):
        return apply_df_hamiltonian(np.asarray(x).reshape(shape), ham, norb, nelec).reshape(-1)

    op = spla.LinearOperator((n, n), matvec=mv, rmatvec=mv, dtype=np.complex128)
    out = spla.expm_multiply((-1j * time) * op, vec.reshape(-1).astype(np.complex128), traceA=0.0)
    return np.asarray(out).reshape(shape)


def trotter_error(vec: np.ndarray, ham, time: float, norb: int, nelec, n_steps: int, order: int,
                  exact: np.ndarray | None = None) -> float:
    """||psi_Trotter - psi_exact||_2 (Sec. 6.2)."""
    if exact is None:
        exact = evolve_exact(vec, ham, time, norb, nelec)
    approx = simulate_trotter(vec, ham, time, norb, nelec, n_steps=n_steps, order=order)
    return float(np.linalg.norm(approx - exact))


# ---------------------------------------------------------------------------
# Exact evolution under each term
# ---------------------------------------------------------------------------

def evolve_one_body(vec: np.ndarray, h: np.ndarray, t: float, norb: int, nelec) -> np.ndarray:
    """exp(-i t sum h_pq a^dag a): an orbital rotation with U = exp(-i h t) (Table 1, last row)."""
    U = scipy.linalg.expm(-1j * t * np.asarray(h))
    return g.apply_orbital_rotation(vec, U, norb, nelec)


def evolve_two_body(vec: np.ndarray, J: np.ndarray, U: np.ndarray, t: float, norb: int,
                    nelec) -> np.ndarray:
    """exp(-i t 1/2 sum J_pq n^(t)_p n^(t)_q) = script-U(U) DC(J, t) script-U(U)^dag (Sec. 4.5.3).

    The basis rotation script-U(U^dag) is applied first.
    """
    phi = g.apply_orbital_rotation(vec, np.asarray(U).conj().T, norb, nelec)
    phi = g.apply_diag_coulomb_evolution(phi, J, t, norb, nelec)
    return g.apply_orbital_rotation(phi, U, norb, nelec)


def _terms(ham):
    yield ("one", None)
    for t in range(ham.n_terms):
        yield ("two", t)


def _apply_term(vec, ham, term, t, norb, nelec):
    kind, idx = term
    if kind == "one":
        return evolve_one_body(vec, ham.h, t, norb, nelec)
    return evolve_two_body(vec, ham.J[idx], ham.U[idx], t, norb, nelec)


def product_formula_step(vec: np.ndarray, apply_term, n_terms: int, dt: float, order: int = 0) -> np.ndarray:
    """One step of the order-k product formula S_k(dt) for H = H_1 + ... + H_L (Sec. 4.5.3), where
    apply_term(vec, k, t) returns exp(-i t H_{k+1}) vec.

    S_0(t) = e^{-iH_L t} ... e^{-iH_1 t}                          (H_1 applied first)
    S_1(t) = e^{-iH_1 t/2} ... e^{-iH_L t/2} e^{-iH_L t/2} ... e^{-iH_1 t/2}
    S_k(t) = S_{k-1}(u_k t)^2 S_{k-1}((1 - 4 u_k) t) S_{k-1}(u_k t)^2,
    u_k = 1 / (4 - 4^{1/(2k-1)}).
    """
    if order == 0:
        for k in range(n_terms):
            vec = apply_term(vec, k, dt)
        return vec
    if order == 1:
        for k in range(n_terms):
            vec = apply_term(vec, k, dt / 2)
        for k in reversed(range(n_terms)):
            vec = apply_term(vec, k, dt / 2)
        return vec
    u = 1.0 / (4.0 - 4.0 ** (1.0 / (2 * order - 1)))
    for t in (u * dt, u * dt, (1 - 4 * u) * dt, u * dt, u * dt):
        vec = product_formula_step(vec, apply_term, n_terms, t, order - 1)
    return vec


def trotter_step(vec: np.ndarray, ham, dt: float, norb: int, nelec, order: int = 0) -> np.ndarray:
    """One step of S_order(dt) for the DF Hamiltonian: H_1 = the one-body term, then the two-body terms in
    array order (Sec. 4.5.3)."""
    terms = list(_terms(ham))
    return product_formula_step(vec, lambda v, k, t: _apply_term(v, ham, terms[k], t, norb, nelec),
                                len(terms), dt, order)


def simulate_trotter(vec: np.ndarray, ham, time: float, norb: int, nelec, n_steps: int = 1,
                     order: int = 0) -> np.ndarray:
    """exp(-i H T) psi ~ S_order(T / r)^r psi with r = n_steps (Sec. 4.5.3)."""
    dt = time / n_steps
    for _ in range(n_steps):
        vec = trotter_step(vec, ham, dt, norb, nelec, order)
    return vec


# ---------------------------------------------------------------------------
# Diagonal Coulomb Hamiltonian (Eq. diagonal-coulomb-hamiltonian)
# ---------------------------------------------------------------------------
# H = sum_{pq,sigma} h_pq a^dag_{p sigma} a_{q sigma} + 1/2 sum_{pq,sigma tau} J^{sigma tau}_pq n_{p sigma} n_{q tau},
# each J^{sigma tau} real symmetric, J^{beta alpha} = (J^{alpha beta})^T.  Sec. 4.5.3 Trotterizes it as the sum of
# two terms: the one-body term (an orbital rotation by exp(-i t h)) and the two-body term (a diagonal Coulomb
# evolution).  Reading: the one-body term is H_1, applied first.

def apply_diag_coulomb_hamiltonian(vec: np.ndarray, h: np.ndarray, J_aa: np.ndarray, norb: int, nelec,
                                   J_ab: np.ndarray | None = None, J_bb: np.ndarray | None = None) -> np.ndarray:
    """H psi for the diagonal Coulomb Hamiltonian (J_ab or J_bb None: J_aa)."""
    out = g.apply_one_body(vec, h, norb, nelec)
    return out + 0.5 * g.diag_coulomb_angle(norb, nelec, J_aa, J_ab, J_bb) * vec


def simulate_trotter_diag_coulomb(vec: np.ndarray, h: np.ndarray, J_aa: np.ndarray, time: float, norb: int, nelec,
                                  J_ab: np.ndarray | None = None, J_bb: np.ndarray | None = None, n_steps: int = 1,
                                  order: int = 0) -> np.ndarray:
    """exp(-i H T) psi ~ S_order(T / r)^r psi for the diagonal Coulomb Hamiltonian, r = n_steps (Sec. 4.5.3)."""

    def term(v, k, t):
        if k == 0:
            return evolve_one_body(v, h, t, norb, nelec)
        return g.apply_diag_coulomb_evolution(v, J_aa, t, norb, nelec, J_ab=J_ab, J_bb=J_bb)

    dt = time / n_steps
    for _ in range(n_steps):
        vec = product_formula_step(vec, term, 2, dt, order)
    return vec


# ---------------------------------------------------------------------------
# Gradient of an energy through a DF Trotter chain (finite differences)
# ---------------------------------------------------------------------------
# Reading (the paper does not treat this gradient): E = Re <psi_T|H_obs|psi_T>
# with psi_T = S_0(dt)^r psi_0 under the evolution Hamiltonian (h, J_t, U_t) and
# a fixed observable H_obs.  Parameters: h and every J_t as symmetric matrices
# (a pair (p, q), p < q, moves both entries), and every U_t through a generator,
# U_t -> U_t expm(A - A^dag) at A = 0 with Re A and Im A entries as parameters.

def df_chain_energy(vec0: np.ndarray, ham, obs, dt: float, n_steps: int, norb: int, nelec) -> float:
    """Re <psi_T|H_obs|psi_T>, psi_T = S_0(dt)^n_steps psi_0."""
    psi = simulate_trotter(vec0, ham, dt * n_steps, norb, nelec, n_steps=n_steps, order=0)
    return float(np.real(df_energy(psi, obs, norb, nelec)))


def _with(ham, h=None, J=None, U=None):
    return type(ham)(h=ham.h if h is None else h, J=ham.J if J is None else J, U=ham.U if U is None else U)


def df_chain_grad_fd(vec0: np.ndarray, ham, obs, dt: float, n_steps: int, norb: int, nelec,
                     step: float = 1e-5) -> dict:
    """Central differences of df_chain_energy: {'h': (N, N) symmetric-pair derivatives,
    'J': (L, N, N) likewise, 'U': (L, 2, N, N) with [t, 0] = d/d Re A, [t, 1] = d/d Im A}."""
    N, L = norb, ham.J.shape[0]

    def E(hh):
        return df_chain_energy(vec0, hh, obs, dt, n_steps, norb, nelec)

    def sym(p, q):
        M = np.zeros((N, N))
        M[p, q] = 1.0
        M[q, p] = 1.0
        return M

    gh = np.zeros((N, N))
    gJ = np.zeros((L, N, N))
    gU = np.zeros((L, 2, N, N))
    for p in range(N):
        for q in range(p, N):
            M = sym(p, q)
            gh[p, q] = gh[q, p] = (E(_with(ham, h=ham.h + step * M)) - E(_with(ham, h=ham.h - step * M))) / (2 * step)
            for t in range(L):
                Jp, Jm = ham.J.copy(), ham.J.copy()
                Jp[t] = Jp[t] + step * M
                Jm[t] = Jm[t] - step * M
                gJ[t, p, q] = gJ[t, q, p] = (E(_with(ham, J=Jp)) - E(_with(ham, J=Jm))) / (2 * step)
    for t in range(L):
        for part in range(2):
            for p in range(N):
                for q in range(N):
                    A = np.zeros((N, N), dtype=complex)
                    A[p, q] = step if part == 0 else 1j * step
                    K = A - A.conj().T
                    Up, Um = ham.U.copy(), ham.U.copy()
                    Up[t] = Up[t] @ scipy.linalg.expm(K)
                    Um[t] = Um[t] @ scipy.linalg.expm(-K)
                    gU[t, part, p, q] = (E(_with(ham, U=Up)) - E(_with(ham, U=Um))) / (2 * step)
    return {"h": gh, "J": gJ, "U": gU}
