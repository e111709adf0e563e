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
