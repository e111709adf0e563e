"""Local unitary cluster Jastrow (LUCJ) ansatz, its energy and its gradient (Sec. 4.5.1).

One repetition is script-U D script-U^dag (Sec. 4.5.1): an orbital rotation, a
diagonal Coulomb evolution, and the inverse rotation, applied to the
Hartree-Fock state, with repetition 1 applied first:

    psi(theta) = prod_{k = n_reps..1} [ script-U(U_k) D_k script-U(U_k)^dag ] |HF>.

Reading of the parameterisation (the paper does not spell it out):
per repetition the flat real vector holds
    [Re A (norb^2, row-major), Im A (norb^2), j_same (norb-1), j_opp (norb)],
K = A - A^dag, U = expm(K), the same U for both spins, and D_k is the diagonal
Coulomb evolution with t = 1, J^{aa} = J^{bb} holding j_same[p] at (p, p+1) and
(p+1, p), J^{ab} = diag(j_opp).  There is no final orbital rotation.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from . import gates as g
from . import hamiltonian as ham_mod
from . import strings as st


def n_params(norb: int, n_reps: int) -> int:
    return n_reps * (2 * norb * norb + 2 * norb - 1)


def unpack(params: np.ndarray, norb: int, n_reps: int):
    """-> list of (K, J_same_matrix, J_opp_matrix) per repetition."""
    per = 2 * norb * norb + 2 * norb - 1
    out = []
    for k in range(n_reps):
        th = params[k * per:(k + 1) * per]
        A = th[:norb * norb].reshape(norb, norb) + 1j * th[norb * norb:2 * norb * norb].reshape(norb, norb)
        js = th[2 * norb * norb:2 * norb * norb + norb - 1]
        jo = th[2 * norb * norb + norb - 1:]
        K = A - A.conj().T
        Jsame = np.zeros((norb, norb))
        for p in range(norb - 1):
            Jsame[p, p + 1] = Jsame[p + 1, p] = js[p]
        Jopp = np.diag(jo)
        out.append((K, Jsame, Jopp))
    return out


def _diag_gate(norb, nelec, Jsame, Jopp):
    """D = exp(-(i/2) sum_{(p,q) in S} J^{sigma tau}_pq) with t = 1."""
    ang = g.diag_coulomb_angle(norb, nelec, Jsame, Jopp, Jsame)
    return np.exp(-0.5j * ang)


def gate_list(params, norb, nelec, n_reps):
    """Gates in application order: ('rot', U) or ('diag', phase-array)."""
    gates = []
    for K, Js, Jo in unpack(params, norb, n_reps):
        U = scipy.linalg.expm(K)
        gates.append(("rot", U.conj().T))
        gates.append(("diag", _diag_gate(norb, nelec, Js, Jo)))
        gates.append(("rot", U))
    return gates


def apply_lucj(params, norb: int, nelec, n_reps: int) -> np.ndarray:
    na, nb = nelec
    vec = np.zeros((st.dim(norb, na), st.dim(norb, nb)), dtype=np.complex128)
    vec[0, 0] = 1.0
    for kind, G in gate_list(params, norb, nelec, n_reps):
        vec = g.apply_orbital_rotation(vec, G, norb, nelec) if kind == "rot" else G * vec
    return vec


def energy(params, ham, norb: int, nelec, n_reps: int) -> float:
    psi = apply_lucj(params, norb, nelec, n_reps)
    return float(np.real(ham_mod.df_energy(psi, ham, norb, nelec)))


def grad_fd(params, ham, norb: int, nelec, n_reps: int, idx=None, h: float = 1e-5) -> np.ndarray:
    """Central finite differences (E(theta + h e_j) - E(theta - h e_j)) / 2h."""
    idx = range(len(params)) if idx is None else idx
    out = []
    for j in idx:
        e = np.zeros_like(params)
        e[j] = h
        out.append((energy(params + e, ham, norb, nelec, n_reps)
                    - energy(params - e, ham, norb, nelec, n_reps)) / (2 * h))
    return np.array(out)


def grad_adjoint(params, ham, norb: int, nelec, n_reps: int):
    """Energy and gradient by the adjoint method; returns (E, grad).

    dE/dtheta = 2 Re <lambda| d psi / d theta>, lambda = H psi.  Walking the gates
    backwards with the costate lambda_i (the costate pulled back through the
    gates after gate i) and the state psi_{i-1} before gate i:
      * diagonal gate D = exp(-i phi): dE/dj = 2 Re sum_I conj(lambda_i) (-i dphi/dj) psi_i,
        psi_i = D psi_{i-1};
      * script-U(U), U = expm(K): U(theta + d) = U e^{d X}, X = U^dag expm_frechet(K, dK),
        so d script-U = script-U(U) X^, X^ = sum X_pq sum_sigma a^dag_p a_q, giving
        2 Re sum_pq X_pq <lambda_{i-1}| E_pq |psi_{i-1}>;
      * script-U(U^dag): U^dag(theta + d) = e^{-d X} U^dag, giving
        -2 Re sum_pq X_pq <lambda_i| E_pq |psi_i>.
    """
    na, nb = nelec
    per = 2 * norb * norb + 2 * norb - 1
    reps = unpack(params, norb, n_reps)
    gates = gate_list(params, norb, nelec, n_reps)
    # forward, keeping every intermediate state (plain, no uncomputation)
    states = []
    vec = np.zeros((st.dim(norb, na), st.dim(norb, nb)), dtype=np.complex128)
    vec[0, 0] = 1.0
    states.append(vec)
    for kind, G in gates:
        vec = g.apply_orbital_rotation(vec, G, norb, nelec) if kind == "rot" else G * vec
        states.append(vec)
    lam = ham_mod.apply_df_hamiltonian(vec, ham, norb, nelec)
    E = float(np.real(np.vdot(vec, lam)))
    grad = np.zeros(len(params))
    xa = st.occupations(norb, na)
    xb = st.occupations(norb, nb)
    # costate after each gate, walking backwards
    lam_after = [None] * len(gates)
    lam_cur = lam
    for i in range(len(gates) - 1, -1, -1):
        lam_after[i] = lam_cur
        kind, G = gates[i]
        lam_cur = g.apply_orbital_rotation(lam_cur, G.conj().T, norb, nelec) if kind == "rot" \
            else np.conj(G) * lam_cur
    for k, (K, Js, Jo) in enumerate(reps):
        base = k * per
        i_udag, i_d, i_u = 3 * k, 3 * k + 1, 3 * k + 2
        U = scipy.linalg.expm(K)
        # transition matrices at the two insertion points
        lam_before_u = g.apply_orbital_rotation(lam_after[i_u], U.conj().T, norb, nelec)
        T_u = g.transition_one_body(lam_before_u, states[i_u], norb, nelec)     # before script-U(U)
        T_udag = g.transition_one_body(lam_after[i_udag], states[i_udag + 1], norb, nelec)  # after script-U(U^dag)
        for part in range(2):
            for p in range(norb):
                for q in range(norb):
                    dA = np.zeros((norb, norb), dtype=np.complex128)
                    dA[p, q] = 1.0 if part == 0 else 1j
                    dK = dA - dA.conj().T
                    L = scipy.linalg.expm_frechet(K, dK, compute_expm=False)
                    X = U.conj().T @ L
                    val = 2 * np.real(np.sum(X * T_u)) - 2 * np.real(np.sum(X * T_udag))
                    grad[base + part * norb * norb + p * norb + q] = val
        # diagonal gate: phi = 1/2 sum_S J, derivative per parameter
        lam_d = lam_after[i_d]
        psi_d = states[i_d + 1]
        w = np.conj(lam_d) * psi_d
        for p in range(norb - 1):
            occ = (xa[:, p] * xa[:, p + 1])[:, None] + (xb[:, p] * xb[:, p + 1])[None, :]
            # j_same[p] enters S twice per spin ((p,p+1) and (p+1,p)), times 1/2
            grad[base + 2 * norb * norb + p] = 2 * np.real(np.sum(w * (-1j) * occ))
        for p in range(norb):
            occ = xa[:, p][:, None] * xb[:, p][None, :]
            # j_opp[p] enters S twice ((p_a, p_b) and (p_b, p_a)), times 1/2
            grad[base + 2 * norb * norb + norb - 1 + p] = 2 * np.real(np.sum(w * (-1j) * occ))
    return E, grad
