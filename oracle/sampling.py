"""Sampling of configurations (Sec. 4.5.4 and 6.1).  Test infrastructure only.

* sample_state: inverse of the cumulative distribution |gamma|^2 in address
  order (alpha-major), one uniform per sample.
* sample_slater: per spin, the orbitals of p(I) = |det U[I, occ]|^2 drawn one at
  a time; the weight of orbital j given the set S drawn so far is the ratio
  det K[S+j, S+j] / det K[S, S] of principal minors of K = Q Q^dag, Q = U[:, occ]
  (the chain rule of this determinantal distribution), and orbital j is the
  first, in orbital order, whose cumulative weight exceeds u_k times the total.
"""
from __future__ import annotations

import numpy as np


def sample_state(vec: np.ndarray, u: np.ndarray) -> np.ndarray:
    """Addresses i_a * dim_b + i_b: the first whose cumulative |gamma|^2 exceeds u * total."""
    p = np.abs(np.asarray(vec).reshape(-1)) ** 2
    cdf = np.cumsum(p)
    idx = np.searchsorted(cdf, np.asarray(u) * cdf[-1], side="right")
    last = int(np.flatnonzero(p)[-1])
    return np.minimum(idx, last).astype(np.int64)


def slater_kernel(U: np.ndarray, occ) -> np.ndarray:
    Q = np.asarray(U)[:, sorted(occ)]
    return Q @ Q.conj().T


def conditional_weights(K: np.ndarray, S: list) -> np.ndarray:
    """w_j = det K[S+j, S+j] / det K[S, S] for j not in S (0 for j in S)."""
    N = K.shape[0]
    base = np.linalg.det(K[np.ix_(S, S)]).real if S else 1.0
    w = np.zeros(N)
    for j in range(N):
        if j in S:
            continue
        T = S + [j]
        w[j] = max(np.linalg.det(K[np.ix_(T, T)]).real / base, 0.0)
    return w


def sample_slater_spin(U: np.ndarray, occ, u_row) -> int:
    """One configuration (bit mask) of one spin for the uniforms u_row (one per electron)."""
    K = slater_kernel(U, occ)
    S = []
    for k in range(len(occ)):
        w = conditional_weights(K, S)
        tot = 0.0
        for x in w:
            tot += x
        target = u_row[k] * tot
        cum, first, last = 0.0, -1, -1
        for j, x in enumerate(w):
            if x > 0:
                cum += x
                last = j
                if first < 0 and cum > target:
                    first = j
        S.append(first if first >= 0 else last)
    return sum(1 << j for j in S)


def sample_slater(norb: int, nelec, U_a, u_a, U_b=None, u_b=None, occ_a=None, occ_b=None):
    """(masks_a, masks_b) for the uniforms u_a (n_samples x n_alpha) and u_b (n_samples x n_beta)."""
    na, nb = nelec
    occ_a = list(range(na)) if occ_a is None else list(occ_a)
    occ_b = list(range(nb)) if occ_b is None else list(occ_b)
    U_b = U_a if U_b is None else U_b
    u_a, u_b = np.asarray(u_a), np.asarray(u_b)
    n_samples = u_a.shape[0]  # u_a, u_b: (n_samples, n_alpha), (n_samples, n_beta); an empty spin gives 0
    ma = np.array([sample_slater_spin(U_a, occ_a, u_a[k]) if na else 0 for k in range(n_samples)], dtype=np.uint64)
    mb = np.array([sample_slater_spin(U_b, occ_b, u_b[k]) if nb else 0 for k in range(n_samples)], dtype=np.uint64)
    return ma, mb
