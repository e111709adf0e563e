"""Brute-force Fock-space reference on 2^(2N) basis states (Jordan-Wigner), for tiny N.

Independent of oracle/: the sector basis is built by multiplying creation
operator matrices onto the vacuum, exactly as |I_a, I_b> = cre_b(I_b) cre_a(I_a)|vac>
is defined (Sec. 2.2, 2.4), and every gate is exp() of its generator as listed
in Table 1.  The only shared object is the list of configurations' ordering,
which this module re-derives itself (ascending integer order of bit masks).
"""
from __future__ import annotations

from itertools import combinations

import numpy as np
import scipy.linalg


class Fock:
    """Spin orbitals: alpha p -> mode p, beta p -> mode norb + p."""

    def __init__(self, norb: int):
        self.norb = norb
        self.nmodes = 2 * norb
        self.dim = 1 << self.nmodes
        self.cre = [self._creation(m) for m in range(self.nmodes)]
        self.ann = [c.conj().T for c in self.cre]

    def _creation(self, m: int) -> np.ndarray:
        # a^dag_m = sigma^+_m (x) prod_{k > m} Z_k on bit strings
        a = np.zeros((self.dim, self.dim))
        for b in range(self.dim):
            if (b >> m) & 1:
                continue
            sign = -1.0 if bin(b >> (m + 1)).count("1") % 2 else 1.0
            a[b | (1 << m), b] = sign
        return a

    def mode(self, p: int, spin: int) -> int:
        return p + spin * self.norb

    def E(self, p: int, q: int) -> np.ndarray:
        """sum_sigma a^dag_{p sigma} a_{q sigma}."""
        return sum(self.cre[self.mode(p, s)] @ self.ann[self.mode(q, s)] for s in (0, 1))

    def n(self, p: int, spin: int) -> np.ndarray:
        m = self.mode(p, spin)
        return self.cre[m] @ self.ann[m]

    def strings(self, n: int):
        masks = sorted(sum(1 << p for p in c) for c in combinations(range(self.norb), n))
        return masks

    def sector_basis(self, nelec) -> np.ndarray:
        """Columns are cre_b(I_b) cre_a(I_a)|vac>, alpha-major over (I_a, I_b)."""
        na, nb = nelec
        vac = np.zeros(self.dim)
        vac[0] = 1.0
        cols = []
        for ma in self.strings(na):
            va = vac.copy()
            for p in range(self.norb):           # ascending right to left: lowest first
                if (ma >> p) & 1:
                    va = self.cre[self.mode(p, 0)] @ va
            for mb in self.strings(nb):
                v = va.copy()
                for p in range(self.norb):
                    if (mb >> p) & 1:
                        v = self.cre[self.mode(p, 1)] @ v
                cols.append(v)
        return np.array(cols).T

    def restrict(self, op: np.ndarray, nelec) -> np.ndarray:
        B = self.sector_basis(nelec)
        return B.T @ op @ B

    # --- gates of Table 1 as exponentials of their generators ---------------
    def orbital_rotation(self, U: np.ndarray, U_b: np.ndarray | None = None) -> np.ndarray:
        La = scipy.linalg.logm(U)
        Lb = La if U_b is None else scipy.linalg.logm(U_b)
        gen = np.zeros((self.dim, self.dim), dtype=complex)
        for p in range(self.norb):
            for q in range(self.norb):
                gen += La[p, q] * self.cre[self.mode(p, 0)] @ self.ann[self.mode(q, 0)]
                gen += Lb[p, q] * self.cre[self.mode(p, 1)] @ self.ann[self.mode(q, 1)]
        return scipy.linalg.expm(gen)

    def one_body(self, M: np.ndarray) -> np.ndarray:
        return sum(M[p, q] * self.E(p, q) for p in range(self.norb) for q in range(self.norb))

    def num_op_sum_gen(self, lam_a, lam_b) -> np.ndarray:
        return sum(lam_a[p] * self.n(p, 0) + lam_b[p] * self.n(p, 1) for p in range(self.norb))

    def diag_coulomb_gen(self, J_aa, J_ab, J_bb) -> np.ndarray:
        """1/2 sum_{pq, sigma tau} J^{sigma tau}_pq n_{p sigma} n_{q tau}, J^{ba} = (J^{ab})^T."""
        blocks = {(0, 0): J_aa, (0, 1): J_ab, (1, 0): J_ab.T, (1, 1): J_bb}
        out = np.zeros((self.dim, self.dim))
        for (s, t), J in blocks.items():
            for p in range(self.norb):
                for q in range(self.norb):
                    out += 0.5 * J[p, q] * self.n(p, s) @ self.n(q, t)
        return out

    def rotated_number(self, U: np.ndarray, p: int, spin: int) -> np.ndarray:
        """n^(t)_{p sigma} = sum_ij U_ip a^dag_{i sigma} a_{j sigma} U*_jp."""
        out = np.zeros((self.dim, self.dim), dtype=complex)
        for i in range(self.norb):
            for j in range(self.norb):
                out += U[i, p] * np.conj(U[j, p]) * (self.cre[self.mode(i, spin)] @ self.ann[self.mode(j, spin)])
        return out

    def df_hamiltonian(self, h, Js, Us) -> np.ndarray:
        H = self.one_body(h).astype(complex)
        for J, U in zip(Js, Us):
            nr = [[self.rotated_number(U, p, s) for p in range(self.norb)] for s in (0, 1)]
            for s in (0, 1):
                for t in (0, 1):
                    for p in range(self.norb):
                        for q in range(self.norb):
                            H += 0.5 * J[p, q] * nr[s][p] @ nr[t][q]
        return H


def to_matrix(vec_sector: np.ndarray, dim_a: int, dim_b: int) -> np.ndarray:
    return vec_sector.reshape(dim_a, dim_b)
