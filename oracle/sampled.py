"""Single amplitudes of a rotated state, for sizes where the full compound matrix is too large.

Gamma'[i, j] = sum_{k, l} C_a[i, k] Gamma[k, l] C_b[j, l] with C_n(U)[J, I] = det U[J, I]
(the same definition as gates.apply_orbital_rotation), so one output amplitude
needs one row of each compound matrix: dim determinants per spin.
"""
from __future__ import annotations

import numpy as np

from . import strings as st


def compound_row(U: np.ndarray, n: int, i: int) -> np.ndarray:
    """Row i of C_n(U): det U[J_i, I] for every n-string I (ascending addresses)."""
    norb = U.shape[0]
    occ = st.occupied_lists(norb, n)
    rows = occ[i]
    sub = np.asarray(U, dtype=np.complex128)[rows[None, :, None], occ[:, None, :]]
    return np.linalg.det(sub)


def rotated_amplitudes(vec: np.ndarray, U_a: np.ndarray, norb: int, nelec, idx,
                       U_b: np.ndarray | None = None) -> np.ndarray:
    """Gamma'[i, j] of script-U(U) Gamma for each (i, j) in idx."""
    na, nb = nelec
    if U_b is None:
        U_b = U_a
    out = []
    ca_cache, cb_cache = {}, {}
    for i, j in idx:
        if i not in ca_cache:
            ca_cache[i] = compound_row(U_a, na, i)
        if j not in cb_cache:
            cb_cache[j] = compound_row(U_b, nb, j)
        out.append(ca_cache[i] @ vec @ cb_cache[j])
    return np.array(out)


def rotated_amplitudes_blocked(vec: np.ndarray, U_a: np.ndarray, norb: int, nelec, idx,
                               U_b: np.ndarray | None = None, block: int = 2048) -> np.ndarray:
    """The same amplitudes as rotated_amplitudes, for states too large to upcast whole.

    Gamma'[i, j] = sum_k C_a[i, k] v_j[k] with v_j[k] = sum_l Gamma[k, l] C_b[j, l];
    v_j is formed over blocks of rows of Gamma, each upcast to complex128 on its own.
    """
    na, nb = nelec
    if U_b is None:
        U_b = U_a
    out = np.empty(len(idx), dtype=np.complex128)
    by_col = {}
    for pos, (i, j) in enumerate(idx):
        by_col.setdefault(int(j), []).append((pos, int(i)))
    for j, rows in by_col.items():
        cb = compound_row(U_b, nb, j)
        v = np.empty(vec.shape[0], dtype=np.complex128)
        for k0 in range(0, vec.shape[0], block):
            v[k0:k0 + block] = np.asarray(vec[k0:k0 + block], dtype=np.complex128) @ cb
        for pos, i in rows:
            out[pos] = compound_row(U_a, na, i) @ v
    return out


def one_body_row(h: np.ndarray, norb: int, n: int, mask: int, amap: dict) -> list:
    """Row `mask` of sum_pq h_pq a^dag_p a_q on n-electron strings: the pairs (address of J, coefficient)
    with coefficient = h_pq <mask| a^dag_p a_q |J>, J = mask with p emptied and q filled (J = mask for p = q)."""
    out = []
    for p in range(norb):
        if not (mask >> p) & 1:
            continue
        for q in range(norb):
            if q != p and (mask >> q) & 1:
                continue
            hv = h[p, q]
            if hv == 0:
                continue
            J = (mask & ~(1 << p)) | (1 << q)
            s = st.excitation_sign(J, p, q) if p != q else 1
            out.append((amap[J], hv * s))
    return out


def diag_coulomb_ham_amplitudes(ham, norb: int, nelec, idx, row, col) -> np.ndarray:
    """(H psi)[i, j] for each (i, j) in idx, for a DF Hamiltonian whose two-body terms all have the identity
    basis (a diagonal Coulomb Hamiltonian, Sec. 2.7.3): the one-body rows of both spins and the diagonal
    weight 1/2 x^T J_t x, x = occupations of both spins.  row(i) / col(j) return psi[i, :] / psi[:, j]."""
    na, nb = nelec
    sa, sb = st.strings(norb, na), st.strings(norb, nb)
    ma, mb = st.address_map(norb, na), st.address_map(norb, nb)
    h = np.asarray(ham.h)
    out = []
    for i, j in idx:
        ci, rj = col(j), row(i)
        a, b = int(sa[i]), int(sb[j])
        v = sum(c * ci[k] for k, c in one_body_row(h, norb, na, a, ma))
        v += sum(c * rj[k] for k, c in one_body_row(h, norb, nb, b, mb))
        x = np.array([((a >> p) & 1) + ((b >> p) & 1) for p in range(norb)], dtype=float)
        w = sum(0.5 * x @ np.asarray(ham.J[t]) @ x for t in range(ham.J.shape[0]))
        out.append(v + w * rj[j])
    return np.array(out)
