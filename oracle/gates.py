"""Gates on a fixed-(N_alpha, N_beta) state matrix Gamma (dim_a x dim_b), complex128.

Every gate here is the plain definition written out; no Givens sweeps, no
merging, no fusion.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import strings as st


# ---------------------------------------------------------------------------
# Orbital rotation (Sec. 2.3 and Table 1)
# ---------------------------------------------------------------------------

_WORKERS = 1


def set_workers(n: int) -> None:
    """Spread the rows of large compound matrices over n forked processes (1 = in this process).

    Only the scheduling changes: every entry is the same determinant either way.
    """
    global _WORKERS
    _WORKERS = max(1, int(n))


def compound_matrix(U: np.ndarray, n: int, chunk: int | None = None, rows=None) -> np.ndarray:
    """C_n(U)[J, I] = det U[J, I] over n-subsets J (rows) and I (columns), ascending addresses.

    From the defining relation of an orbital rotation, script-U a^dag_p
    script-U^dag = sum_q U_qp a^dag_q (Sec. 2.3): applying it to
    cre(I)|vac> = a^dag_{i_n}...a^dag_{i_1}|vac> and collecting the ordered
    products gives sum_J det(U[J, I]) |J>, i.e. column I of C_n(U).
    C_0(U) = [[1]].  A real U (no nonzero imaginary part) gives a real matrix,
    its determinants taken in float64.  rows (optional): only those rows J, in
    the order given.
    """
    norb = U.shape[0]
    occ = st.occupied_lists(norb, n)
    d = len(occ)
    U = np.asarray(U)
    real = not np.iscomplexobj(U) or not np.any(U.imag)
    dtype = np.float64 if real else np.complex128
    U = np.ascontiguousarray(U.real if real else U, dtype=dtype)
    if n == 0:
        return np.ones((1, 1), dtype=dtype)
    if chunk is None:
        chunk = max(1, min(256, (1 << 26) // (d * n * n)))

    row_occ = occ if rows is None else occ[np.asarray(rows, dtype=np.int64)]
    nr = len(row_occ)

    def fill(j0, j1, out):
        for a in range(j0, j1, chunk):
            b = min(a + chunk, j1)
            # minors[r, c] = U[row_occ[a + r]][:, occ[c]]  -> shape (b - a, d, n, n)
            sub = U[row_occ[a:b, None, :, None], occ[None, :, None, :]]
            out[a:b] = np.linalg.det(sub)

    if _WORKERS <= 1 or nr < 4 * chunk:
        out = np.empty((nr, d), dtype=dtype)
        fill(0, nr, out)
        return out
    import mmap
    import multiprocessing
    buf = mmap.mmap(-1, nr * d * np.dtype(dtype).itemsize)
    out = np.frombuffer(buf, dtype=dtype).reshape(nr, d)
    bounds = np.linspace(0, nr, _WORKERS + 1).astype(int)
    ctx = multiprocessing.get_context("fork")
    procs = [ctx.Process(target=fill, args=(int(bounds[k]), int(bounds[k + 1]), out))
             for k in range(_WORKERS)]
    for pr in procs:
        pr.start()
    for pr in procs:
        pr.join()
    if any(pr.exitcode != 0 for pr in procs):
        raise RuntimeError("compound_matrix: a worker process failed")
    return out


def _sandwich(Ca: np.ndarray, vec: np.ndarray, Cb: np.ndarray) -> np.ndarray:
    """Ca vec Cb^T; with real compound matrices the real and imaginary parts of vec go separately."""
    if Ca.dtype == np.float64 and Cb.dtype == np.float64:
        re = Ca @ np.ascontiguousarray(vec.real) @ Cb.T
        im = Ca @ np.ascontiguousarray(vec.imag) @ Cb.T
        out = np.empty(re.shape, dtype=np.complex128)
        out.real = re
        out.imag = im
        return out
    return Ca @ vec @ Cb.T


def apply_orbital_rotation(vec: np.ndarray, U_a: np.ndarray, norb: int, nelec,
                           U_b: np.ndarray | None = None) -> np.ndarray:
    """script-U(U) = exp(sum_pq log(U)_pq a^dag_p a_q) on both spins (Sec. 2.3, 3.2.3).

    Gamma' = C_{n_a}(U_a) Gamma C_{n_b}(U_b)^T (transpose, not dagger: the beta
    index is the column index).  U_b = None means the same U for both spins.
    """
    na, nb = nelec
    same = U_b is None or U_b is U_a
    Ca = compound_matrix(np.asarray(U_a), na)
    Cb = Ca if (same and na == nb) else compound_matrix(np.asarray(U_a if U_b is None else U_b), nb)
    return _sandwich(Ca, np.asarray(vec, dtype=np.complex128), Cb)


# ---------------------------------------------------------------------------
# Number-operator-sum evolution (Sec. 3.2.1)
# ---------------------------------------------------------------------------

def apply_num_op_sum_evolution(vec: np.ndarray, lam_a: np.ndarray, time: float, norb: int,
                               nelec, lam_b: np.ndarray | None = None) -> np.ndarray:
    """gamma' = exp(-i t (sum_{p in I_a} lam_a[p] + sum_{p in I_b} lam_b[p])) gamma."""
    na, nb = nelec
    if lam_b is None:
        lam_b = lam_a
    xa = st.occupations(norb, na)
    xb = st.occupations(norb, nb)
    ang = (xa @ np.asarray(lam_a, float))[:, None] + (xb @ np.asarray(lam_b, float))[None, :]
    return np.exp(-1j * time * ang) * vec


# ---------------------------------------------------------------------------
# Diagonal Coulomb evolution (Sec. 3.2.2)
# ---------------------------------------------------------------------------

def diag_coulomb_angle(norb: int, nelec, J_aa: np.ndarray, J_ab: np.ndarray | None = None,
                       J_bb: np.ndarray | None = None) -> np.ndarray:
    """sum over the multiset S of (p, q) pairs of J^{sigma tau}_pq, per configuration.

    S holds (p in I_a, q in I_a), (p in I_a, q in I_b), (p in I_b, q in I_a),
    (p in I_b, q in I_b), diagonal p = q included.  The (b, a) block uses
    J^{ba} = (J^{ab})^T.  A single matrix fills all blocks.
    Returns a (dim_a, dim_b) array of sum_{(p,q) in S} J_pq.
    """
    na, nb = nelec
    if J_ab is None:
        J_ab = J_aa
    if J_bb is None:
        J_bb = J_aa
    xa = st.occupations(norb, na)
    xb = st.occupations(norb, nb)
    aa = np.einsum("ip,pq,iq->i", xa, J_aa, xa)
    bb = np.einsum("ip,pq,iq->i", xb, J_bb, xb)
    ab = xa @ J_ab @ xb.T          # p in I_a, q in I_b
    ba = (xb @ J_ab.T @ xa.T).T    # p in I_b, q in I_a with J^{ba} = (J^{ab})^T
    return aa[:, None] + bb[None, :] + ab + ba


def diag_coulomb_angle_at(norb: int, nelec, idx, J_aa: np.ndarray, J_ab: np.ndarray | None = None,
                          J_bb: np.ndarray | None = None) -> np.ndarray:
    """diag_coulomb_angle evaluated only at the (i_a, i_b) address pairs in idx.

    The same multiset sum, x_a J^{aa} x_a + x_a J^{ab} x_b + x_b J^{ba} x_a
    + x_b J^{bb} x_b, for states too large for the whole (dim_a, dim_b) table.
    """
    na, nb = nelec
    if J_ab is None:
        J_ab = J_aa
    if J_bb is None:
        J_bb = J_aa
    idx = np.asarray(idx)
    xa = st.occupations(norb, na)[idx[:, 0]]
    xb = st.occupations(norb, nb)[idx[:, 1]]
    aa = np.einsum("ip,pq,iq->i", xa, J_aa, xa)
    bb = np.einsum("ip,pq,iq->i", xb, J_bb, xb)
    ab = np.einsum("ip,pq,iq->i", xa, J_ab, xb)
    ba = np.einsum("ip,pq,iq->i", xb, np.asarray(J_ab).T, xa)
    return aa + bb + ab + ba


def apply_diag_coulomb_evolution(vec: np.ndarray, J: np.ndarray, time: float, norb: int, nelec,
                                 J_ab: np.ndarray | None = None,
                                 J_bb: np.ndarray | None = None) -> np.ndarray:
    """gamma' = exp(-(1/2) i t sum_{(p,q) in S} J_pq) gamma (Sec. 3.2.2).

    With only J given, J^{aa} = J^{ab} = J^{bb} = J.
    """
    ang = diag_coulomb_angle(norb, nelec, J, J_ab, J_bb)
    return np.exp(-0.5j * time * ang) * vec


# ---------------------------------------------------------------------------
# Givens pair action (Sec. 3.2.3)
# ---------------------------------------------------------------------------

def apply_givens(vec: np.ndarray, c: float, s: complex, p: int, q: int, norb: int, nelec,
                 spin: int) -> np.ndarray:
    """The Givens rotation [[c, s], [-s*, c]] on orbitals (p, q) of one spin.

    For each configuration I with p in I, q not in I and I' = I^{p->q}:
      gamma'(I) = c gamma(I) + eps s gamma(I'),  gamma'(I') = -eps s* gamma(I) + c gamma(I'),
    where eps = (-1)^(number of occupied orbitals strictly between p and q).
    The paper's formula omits eps; it is exact as printed for adjacent orbitals
    (eps = 1), which is the only case the rotation networks use.
    """
    n = nelec[spin]
    s_list = st.strings(norb, n)
    amap = st.address_map(norb, n)
    out = vec.copy()
    for i, m in enumerate(s_list):
        m = int(m)
        if (m >> p) & 1 and not (m >> q) & 1:
            m2 = (m & ~(1 << p)) | (1 << q)
            j = amap[m2]
            eps = st.excitation_sign(m, q, p)
            if spin == 0:
                x, y = vec[i, :], vec[j, :]
                out[i, :] = c * x + eps * s * y
                out[j, :] = -eps * np.conj(s) * x + c * y
            else:
                x, y = vec[:, i], vec[:, j]
                out[:, i] = c * x + eps * s * y
                out[:, j] = -eps * np.conj(s) * x + c * y
    return out


# ---------------------------------------------------------------------------
# One-body excitation operators E^sigma_pq = a^dag_{p sigma} a_{q sigma}
# ---------------------------------------------------------------------------

def excitation_matrix(norb: int, n: int, p: int, q: int) -> sp.csr_matrix:
    """Sparse dim x dim matrix of a^dag_p a_q on n-electron strings of one spin."""
    s_list = st.strings(norb, n)
    amap = st.address_map(norb, n)
    rows, cols, vals = [], [], []
    for i, m in enumerate(s_list):
        m = int(m)
        if not (m >> q) & 1:
            continue
        if p != q and (m >> p) & 1:
            continue
        m2 = (m & ~(1 << q)) | (1 << p)
        rows.append(amap[m2])
        cols.append(i)
        vals.append(float(st.excitation_sign(m, p, q)) if p != q else 1.0)
    d = len(s_list)
    return sp.csr_matrix((vals, (rows, cols)), shape=(d, d), dtype=np.complex128)


def one_body_matrix(M: np.ndarray, norb: int, n: int) -> sp.csr_matrix:
    """sum_pq M_pq a^dag_p a_q restricted to n-electron strings of one spin."""
    d = st.dim(norb, n)
    out = sp.csr_matrix((d, d), dtype=np.complex128)
    for p in range(norb):
        for q in range(norb):
            if M[p, q] != 0:
                out = out + M[p, q] * excitation_matrix(norb, n, p, q)
    return out


def apply_one_body(vec: np.ndarray, M: np.ndarray, norb: int, nelec) -> np.ndarray:
    """(sum_pq M_pq sum_sigma a^dag_{p sigma} a_{q sigma}) applied to Gamma."""
    na, nb = nelec
    Aa = one_body_matrix(M, norb, na)
    Ab = one_body_matrix(M, norb, nb)
    return Aa @ vec + (Ab @ vec.T).T


def transition_one_body(lam: np.ndarray, vec: np.ndarray, norb: int, nelec) -> np.ndarray:
    """T_pq = <lam| sum_sigma a^dag_{p sigma} a_{q sigma} |vec>, summed over both spins."""
    na, nb = nelec
    T = np.zeros((norb, norb), dtype=np.complex128)
    lc = lam.conj()
    for p in range(norb):
        for q in range(norb):
            Ea = excitation_matrix(norb, na, p, q)
            Eb = excitation_matrix(norb, nb, p, q)
            T[p, q] = np.sum(lc * (Ea @ vec)) + np.sum(lc * (Eb @ vec.T).T)
    return T


# ---------------------------------------------------------------------------
# The remaining gates of Table 1, the Slater determinant (Sec. 2.4) and the
# unitary cluster Jastrow forward pass (Sec. 4.5.1)
# ---------------------------------------------------------------------------

def _spin_occ(norb: int, nelec, spin: int) -> np.ndarray:
    return st.occupations(norb, nelec[spin])


def apply_num_interaction(vec: np.ndarray, theta: float, p: int, spin: int, norb: int, nelec) -> np.ndarray:
    """exp(i theta n_{p sigma}): each configuration times exp(i theta x_sigma[p])."""
    x = _spin_occ(norb, nelec, spin)[:, p]
    f = np.exp(1j * theta * x)
    return vec * (f[:, None] if spin == 0 else f[None, :])


def apply_num_num_interaction(vec: np.ndarray, theta: float, p: int, sigma: int, q: int, tau: int, norb: int,
                              nelec) -> np.ndarray:
    """exp(i theta n_{p sigma} n_{q tau}): each configuration times exp(i theta x_sigma[p] x_tau[q])."""
    xs = [_spin_occ(norb, nelec, 0), _spin_occ(norb, nelec, 1)]
    def col(spin, r):
        v = xs[spin][:, r]
        return v[:, None] if spin == 0 else v[None, :]
    return vec * np.exp(1j * theta * col(sigma, p) * col(tau, q))


def _one_spin(vec, U, spin, norb, nelec):
    eye = np.eye(norb, dtype=np.complex128)
    return apply_orbital_rotation(vec, U if spin == 0 else eye, norb, nelec, U_b=U if spin == 1 else eye)


def apply_givens_rotation(vec: np.ndarray, theta: float, p: int, q: int, spin: int, norb: int, nelec) -> np.ndarray:
    """exp(theta (a+_{p s} a_{q s} - a+_{q s} a_{p s})): the orbital rotation of spin s by
    U = expm(K), K = theta (|p><q| - |q><p|) (the generator's one-body matrix)."""
    import scipy.linalg
    K = np.zeros((norb, norb))
    K[p, q], K[q, p] = theta, -theta
    return _one_spin(vec, scipy.linalg.expm(K), spin, norb, nelec)


def apply_tunneling_interaction(vec: np.ndarray, theta: float, p: int, q: int, spin: int, norb: int,
                                nelec) -> np.ndarray:
    """exp(i theta (a+_{p s} a_{q s} + h.c.)): the orbital rotation of spin s by expm(K),
    K = i theta (|p><q| + |q><p|)."""
    import scipy.linalg
    K = np.zeros((norb, norb), dtype=np.complex128)
    K[p, q] = K[q, p] = 1j * theta
    return _one_spin(vec, scipy.linalg.expm(K), spin, norb, nelec)


def apply_quad_ham_evolution(vec: np.ndarray, M: np.ndarray, time: float, norb: int, nelec,
                             M_b: np.ndarray | None = None) -> np.ndarray:
    """exp(-i t sum M^sigma_pq a+_{p sigma} a_{q sigma}) = orbital rotation by expm(-i t M) (Table 1)."""
    import scipy.linalg
    Ua = scipy.linalg.expm(-1j * time * np.asarray(M))
    Ub = Ua if M_b is None else scipy.linalg.expm(-1j * time * np.asarray(M_b))
    return apply_orbital_rotation(vec, Ua, norb, nelec, U_b=Ub)


def slater_determinant(norb: int, nelec, occ_a=None, occ_b=None, U_a=None, U_b=None) -> np.ndarray:
    """script-U(U) |occ>: the orbital rotation applied to the basis state whose occupied orbitals are
    occ_a, occ_b (default: the lowest, Hartree-Fock), Sec. 2.4."""
    na, nb = nelec
    amap_a, amap_b = st.address_map(norb, na), st.address_map(norb, nb)
    occ_a = list(range(na)) if occ_a is None else list(occ_a)
    occ_b = list(range(nb)) if occ_b is None else list(occ_b)
    vec = np.zeros((st.dim(norb, na), st.dim(norb, nb)), dtype=np.complex128)
    vec[amap_a[sum(1 << o for o in occ_a)], amap_b[sum(1 << o for o in occ_b)]] = 1.0
    eye = np.eye(norb, dtype=np.complex128)
    Ua = eye if U_a is None else np.asarray(U_a)
    Ub = Ua if U_b is None else np.asarray(U_b)
    return apply_orbital_rotation(vec, Ua, norb, nelec, U_b=Ub)


def apply_ucj(norb: int, nelec, U_a, J_aa, U_b=None, J_ab=None, J_bb=None, final_a=None,
              final_b=None) -> np.ndarray:
    """[script-U(F)] prod_{k = R..1} script-U(U_k) D_k script-U(U_k)^dag |HF>, D_k the diagonal Coulomb
    evolution at t = 1 with (J_aa[k], J_ab[k], J_bb[k]); gates applied one by one (no merging)."""
    R = len(U_a)
    U_b = U_a if U_b is None else U_b
    J_ab = J_aa if J_ab is None else J_ab
    J_bb = J_aa if J_bb is None else J_bb
    vec = slater_determinant(norb, nelec)
    for k in range(R):
        vec = apply_orbital_rotation(vec, np.asarray(U_a[k]).conj().T, norb, nelec, U_b=np.asarray(U_b[k]).conj().T)
        vec = apply_diag_coulomb_evolution(vec, J_aa[k], 1.0, norb, nelec, J_ab=J_ab[k], J_bb=J_bb[k])
        vec = apply_orbital_rotation(vec, U_a[k], norb, nelec, U_b=U_b[k])
    if final_a is not None:
        vec = apply_orbital_rotation(vec, final_a, norb, nelec, U_b=final_a if final_b is None else final_b)
    return vec


def apply_in_basis(vec: np.ndarray, B: np.ndarray, gate, norb: int, nelec) -> np.ndarray:
    """script-U(B) gate(script-U(B)^dag vec): a diagonal gate in the basis of the rotated orbitals."""
    B = np.asarray(B, dtype=np.complex128)
    phi = apply_orbital_rotation(vec, B.conj().T, norb, nelec)
    return apply_orbital_rotation(gate(phi), B, norb, nelec)
