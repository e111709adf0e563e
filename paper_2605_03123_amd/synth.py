"""Seeded synthetic inputs shared by the oracle tests, the GPU parity tests and the bench.

This module only draws random numbers and shapes them into the objects the
workloads need (states, unitary and orthogonal matrices, symmetric matrices,
parameter vectors).  It performs none of the fermionic-state arithmetic: no
string tables, no gates, no Hamiltonian action.

Conventions (each is a reading of an unstated detail of the paper's random
benchmark objects, Sec. 5.2):
  * "N(0, x)" means standard deviation x (numpy ``scale``).
  * A symmetric matrix with "entries N(0, x)" draws the upper triangle
    including the diagonal iid and mirrors it.
  * Haar unitaries come from QR of a complex Gaussian matrix with the phases of
    R's diagonal moved into Q (Mezzadri's fix); real orthogonal matrices from
    QR of a real Gaussian matrix with the signs of R's diagonal moved into Q.
  * Complex Gaussians have iid N(0, 1) real and imaginary parts.
  * Every generator takes a ``numpy.random.Generator``; the workloads below use
    ``numpy.random.default_rng(seed)`` (PCG64) with a fixed draw order.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from math import comb

import numpy as np


def rng(seed) -> np.random.Generator:
    return np.random.default_rng(seed)


def random_state(r: np.random.Generator, dim_a: int, dim_b: int) -> np.ndarray:
    """iid complex Gaussian dim_a x dim_b matrix, normalised in FP64."""
    v = r.standard_normal((dim_a, dim_b)) + 1j * r.standard_normal((dim_a, dim_b))
    v /= np.linalg.norm(v)
    return v


def random_unitary(r: np.random.Generator, n: int) -> np.ndarray:
    """Haar-random n x n unitary (QR with phases fixed)."""
    z = r.standard_normal((n, n)) + 1j * r.standard_normal((n, n))
    q, rr = np.linalg.qr(z)
    d = np.diagonal(rr)
    return q * (d / np.abs(d))


def random_orthogonal(r: np.random.Generator, n: int) -> np.ndarray:
    """Haar-random n x n real orthogonal matrix (QR with signs fixed)."""
    z = r.standard_normal((n, n))
    q, rr = np.linalg.qr(z)
    return q * np.sign(np.diagonal(rr))


def random_symmetric(r: np.random.Generator, n: int, scale: float) -> np.ndarray:
    """Real symmetric matrix, upper triangle (with diagonal) iid N(0, scale)."""
    m = np.zeros((n, n))
    iu = np.triu_indices(n)
    m[iu] = r.normal(0.0, scale, size=len(iu[0]))
    return m + np.triu(m, 1).T


def random_hermitian(r: np.random.Generator, n: int, scale: float) -> np.ndarray:
    z = r.normal(0.0, scale, (n, n)) + 1j * r.normal(0.0, scale, (n, n))
    return 0.5 * (z + z.conj().T)


@dataclass
class DFHamiltonian:
    """Double-factorized Hamiltonian data (Eq. double-factorized-hamiltonian).

    h: (norb, norb) real symmetric one-body matrix.
    J: (L, norb, norb) real symmetric diagonal-Coulomb matrices.
    U: (L, norb, norb) unitary (here real orthogonal) basis rotations.
    """

    h: np.ndarray
    J: np.ndarray
    U: np.ndarray

    @property
    def norb(self) -> int:
        return self.h.shape[0]

    @property
    def n_terms(self) -> int:
        return self.J.shape[0]


def df_hamiltonian(r: np.random.Generator, norb: int, n_terms: int,
                   h_scale: float = 0.5, j_scale: float = 0.1) -> DFHamiltonian:
    """h ~ sym N(0, h_scale); per term: U_t real orthogonal (QR), J_t ~ sym N(0, j_scale).

    Draw order: h, then for each term U_t followed by J_t.
    """
    h = random_symmetric(r, norb, h_scale)
    Us, Js = [], []
    for _ in range(n_terms):
        Us.append(random_orthogonal(r, norb))
        Js.append(random_symmetric(r, norb, j_scale))
    return DFHamiltonian(h=h, J=np.array(Js), U=np.array(Us, dtype=np.complex128))


def lucj_n_params(norb: int, n_reps: int) -> int:
    """Flat LUCJ parameter count: per rep Re A, Im A (norb^2 each), j_same (norb-1), j_opp (norb)."""
    return n_reps * (2 * norb * norb + 2 * norb - 1)


def lucj_params(r: np.random.Generator, norb: int, n_reps: int, scale: float = 0.1) -> np.ndarray:
    return r.normal(0.0, scale, size=lucj_n_params(norb, n_reps))


def dim(norb: int, n: int) -> int:
    return comb(norb, n)


def hartree_fock(dim_a: int, dim_b: int) -> np.ndarray:
    """The lowest-orbitals configuration sits at address (0, 0) in both spins."""
    v = np.zeros((dim_a, dim_b), dtype=np.complex128)
    v[0, 0] = 1.0
    return v


# ---------------------------------------------------------------------------
# Named workloads (the five synthetic problem shapes the build is measured on)
# ---------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    norb: int
    nelec: tuple
    data: dict = field(default_factory=dict)


def workload_rotation_coulomb(seed: int = 0) -> Workload:
    """norb=8, (4,4): random state, Haar U, J ~ sym N(0,1), t = 0.3.

    Draw order: state, U, J.
    """
    norb, nelec = 8, (4, 4)
    r = rng(seed)
    da, db = dim(norb, 4), dim(norb, 4)
    vec = random_state(r, da, db)
    U = random_unitary(r, norb)
    J = random_symmetric(r, norb, 1.0)
    return Workload("rotation+diag_coulomb n8 (4,4)", norb, nelec,
                    dict(vec=vec, U=U, J=J, t=0.3))


def workload_df_trotter(norb: int, n_terms: int, seed: int = 0, start: str = "hf",
                        dt: float = 0.1, n_steps: int = 1) -> Workload:
    """DF Hamiltonian (h ~ N(0,0.5), L terms with U_t orthogonal, J_t ~ N(0,0.1)).

    Draw order: Hamiltonian, then the start state if random.
    """
    n = norb // 2
    r = rng(seed)
    ham = df_hamiltonian(r, norb, n_terms)
    da = db = dim(norb, n)
    if start == "hf":
        vec = hartree_fock(da, db)
    else:
        vec = random_state(r, da, db)
    return Workload(f"df_trotter n{norb} ({n},{n}) L{n_terms}", norb, (n, n),
                    dict(ham=ham, vec=vec, dt=dt, n_steps=n_steps))


def workload_lucj(norb: int, n_reps: int, n_terms: int, seed: int = 0,
                  nelec: tuple | None = None) -> Workload:
    """LUCJ parameters N(0, 0.1) and a DF Hamiltonian with n_terms terms.

    Draw order: parameters, then Hamiltonian.
    """
    if nelec is None:
        nelec = (norb // 2, norb // 2)
    r = rng(seed)
    params = lucj_params(r, norb, n_reps)
    ham = df_hamiltonian(r, norb, n_terms)
    return Workload(f"lucj n{norb} {nelec} reps{n_reps} L{n_terms}", norb, nelec,
                    dict(params=params, n_reps=n_reps, ham=ham))


def workload_batched(n_inst: int = 256, seed: int = 0, n_reps: int = 2):
    """Instances with norb in {8,10,12} uniform and n in {norb/2-1, norb/2}.

    Instance i draws from default_rng([seed, i]): norb, n, parameters, Hamiltonian.
    """
    out = []
    for i in range(n_inst):
        r = rng([seed, i])
        norb = int(r.choice([8, 10, 12]))
        n = int(r.choice([norb // 2 - 1, norb // 2]))
        params = lucj_params(r, norb, n_reps)
        ham = df_hamiltonian(r, norb, norb)
        out.append(Workload(f"inst{i}", norb, (n, n), dict(params=params, n_reps=n_reps, ham=ham)))
    return out


def fd_indices(n_params: int, count: int = 20, seed=(0, 1)) -> np.ndarray:
    return np.sort(rng(list(seed)).choice(n_params, count, replace=False))


def lattice_edges(nx: int, ny: int, periodic_x: bool = True, periodic_y: bool = False) -> list:
    """Nearest-neighbour pairs of an nx x ny square lattice, site (x, y) -> x + nx * y.

    A periodic direction adds the wrap-around pair (n - 1, 0); it needs n >= 3,
    so that no pair is listed twice.
    """
    if (periodic_x and nx < 3) or (periodic_y and ny < 3):
        raise ValueError("a periodic direction needs at least 3 sites")
    edges = []
    for y in range(ny):
        for x in range(nx):
            p = x + nx * y
            if x + 1 < nx or periodic_x:
                edges.append((p, (x + 1) % nx + nx * y))
            if y + 1 < ny or periodic_y:
                edges.append((p, x + nx * ((y + 1) % ny)))
    return edges


def hubbard_2d(nx: int, ny: int, t: float = 1.0, U: float = 8.0, periodic_x: bool = True,
               periodic_y: bool = False) -> DFHamiltonian:
    """The 2D Hubbard model H = -t sum_<pq>,s (a+_ps a_qs + h.c.) + U sum_p n_pa n_pb
    (Sec. 6.2) in the double-factorized form the library takes: one term with
    the identity basis and J = U * I, whose 1/2 sum_p U (n_pa + n_pb)^2 equals
    U sum_p n_pa n_pb + (U/2) sum_ps n_ps; the one-body matrix carries -U/2 on
    its diagonal to cancel the second part.  Defaults: the paper's t = 1,
    U = 8, periodic in x only.
    """
    n = nx * ny
    h = np.zeros((n, n))
    for p, q in lattice_edges(nx, ny, periodic_x, periodic_y):
        h[p, q] -= t
        h[q, p] -= t
    h -= 0.5 * U * np.eye(n)
    return DFHamiltonian(h=h, J=(U * np.eye(n))[None], U=np.eye(n, dtype=np.complex128)[None])


def hubbard_2d_diag_coulomb(nx: int, ny: int, t: float = 1.0, U: float = 8.0, periodic_x: bool = True,
                            periodic_y: bool = False):
    """The same 2D Hubbard model as a diagonal Coulomb Hamiltonian (Eq. diagonal-coulomb-hamiltonian), as
    printed: (h, J_aa, J_ab, J_bb) with h the hopping matrix, J_aa = J_bb = 0 and J_ab = U * I, so that
    1/2 sum J^{st}_pq n_ps n_qt = U sum_p n_pa n_pb."""
    n = nx * ny
    h = np.zeros((n, n))
    for p, q in lattice_edges(nx, ny, periodic_x, periodic_y):
        h[p, q] -= t
        h[q, p] -= t
    return h, np.zeros((n, n)), U * np.eye(n), np.zeros((n, n))


def hubbard_filling(nx: int, ny: int, fraction: float = 0.125) -> tuple:
    """(n_alpha, n_beta) for a filling fraction of the 2 nx ny spin orbitals
    (the paper's 1/8 filling: nx ny / 4 electrons), alpha taking the odd one."""
    ne = int(round(2 * nx * ny * fraction))
    return ((ne + 1) // 2, ne // 2)
