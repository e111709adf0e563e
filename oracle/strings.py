"""Electronic configurations (strings) and state-vector addresses.

A configuration of one spin is a subset I of {0..N-1} (Sec. 2.2); it is stored
as the N-bit integer with bit p set when p is in I.  The paper assigns
addresses with PySCF's FCI module (Sec. 3.1) without stating the order; the
reading taken here is ascending integer order of the bit masks (the
combinatorial number system), which puts the Hartree-Fock configuration
{0..n-1} at address 0.  PySCF compatibility of the addresses is parity
unpinned (PySCF is not available).

The state vector for the sector (N_alpha, N_beta) is the dim_a x dim_b matrix
Gamma[i_a, i_b] = gamma(I_alpha, I_beta) (Sec. 3.1), alpha-major.
"""
from __future__ import annotations

from functools import lru_cache
from itertools import combinations
from math import comb

import numpy as np


def dim(norb: int, n: int) -> int:
    """Number of n-electron configurations of one spin, C(N, n) (Sec. 2.6)."""
    return comb(norb, n)


@lru_cache(maxsize=None)
def strings(norb: int, n: int) -> np.ndarray:
    """All n-subsets of {0..norb-1} as int64 bit masks, in ascending integer order."""
    masks = [sum(1 << p for p in c) for c in combinations(range(norb), n)]
    return np.array(sorted(masks), dtype=np.int64)


@lru_cache(maxsize=None)
def address_map(norb: int, n: int) -> dict:
    """mask -> address (index in the sorted list)."""
    return {int(m): i for i, m in enumerate(strings(norb, n))}


def occupations(norb: int, n: int) -> np.ndarray:
    """(dim, norb) 0/1 float matrix: row i is the occupation vector x of string i."""
    s = strings(norb, n)
    return ((s[:, None] >> np.arange(norb)[None, :]) & 1).astype(np.float64)


def occupied_lists(norb: int, n: int) -> np.ndarray:
    """(dim, n) int array: row i lists the occupied orbitals of string i in ascending order."""
    s = strings(norb, n)
    out = np.zeros((len(s), n), dtype=np.int64)
    for i, m in enumerate(s):
        out[i] = [p for p in range(norb) if (int(m) >> p) & 1]
    return out


def excitation_sign(mask: int, p: int, q: int) -> int:
    """Sign of a^dag_p a_q acting on cre(I)|vac> (creators ascending right to left, Sec. 2.2).

    a_q anticommutes past the creators of orbitals above q; a^dag_p is then moved
    into its ordered place past the remaining creators above p.  The result is
    (-1)^(number of occupied orbitals strictly between p and q).
    """
    lo, hi = min(p, q), max(p, q)
    between = (mask >> (lo + 1)) & ((1 << max(hi - lo - 1, 0)) - 1)
    return -1 if bin(between).count("1") % 2 else 1
