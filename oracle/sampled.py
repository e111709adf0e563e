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
