"""Pins for oracle/strings.py: dimensions, ordering, Hartree-Fock address, excitation signs."""
from math import comb

import numpy as np
import pytest

from oracle import strings as st
from jw import Fock


@pytest.mark.parametrize("norb,n", [(1, 0), (1, 1), (4, 2), (8, 4), (10, 3), (12, 6)])
def test_count_and_order(norb, n):
    s = st.strings(norb, n)
    assert len(s) == comb(norb, n)
    assert np.all(np.diff(s) > 0)
    assert all(bin(int(m)).count("1") == n for m in s)


@pytest.mark.parametrize("norb,n", [(6, 3), (9, 4), (12, 5)])
def test_address_is_combinatorial_rank(norb, n):
    # ascending integer order == rank sum_k C(i_k, k) of the combinatorial number system
    occ = st.occupied_lists(norb, n)
    ranks = [sum(comb(int(i), k + 1) for k, i in enumerate(row)) for row in occ]
    assert ranks == list(range(len(occ)))


def test_hartree_fock_is_address_zero():
    for norb, n in [(8, 4), (16, 8), (14, 7)]:
        assert int(st.strings(norb, n)[0]) == (1 << n) - 1


def test_memory_figures_of_the_paper():
    gib, mib = 2.0 ** 30, 2.0 ** 20
    # Sec. 5.2: 16 spatial orbitals, 1/2 filling: 2.5 GiB; 1/4 filling: 51 MiB (complex128)
    assert round(st.dim(16, 8) ** 2 * 16 / gib, 1) == 2.5
    assert round(st.dim(16, 4) ** 2 * 16 / mib) == 51
    # Sec. 1: 4x8 Hubbard (32 orbitals) at 1/8 filling (64 spin orbitals -> 8 electrons): 19.3 GiB
    assert round(st.dim(32, 4) ** 2 * 16 / gib, 1) == 19.3
    # Sec. 6.1: N2 (10e, 26o): 64.5 GiB
    assert round(st.dim(26, 5) ** 2 * 16 / gib, 1) == 64.5
    # Sec. 5.2: 32 qubits would need 64 GiB in a general simulator
    assert 2 ** 32 * 16 / gib == 64


@pytest.mark.parametrize("norb,nelec", [(3, (1, 2)), (3, (2, 2)), (4, (2, 1))])
def test_excitation_sign_matches_fock_space(norb, nelec):
    """<J| a^dag_p a_q |I> from creation-operator matrices equals the oracle's sign rule."""
    from oracle import gates as g
    F = Fock(norb)
    for spin in (0, 1):
        for p in range(norb):
            for q in range(norb):
                op = F.cre[F.mode(p, spin)] @ F.ann[F.mode(q, spin)]
                M = F.restrict(op, nelec)
                da, db = st.dim(norb, nelec[0]), st.dim(norb, nelec[1])
                Es = g.excitation_matrix(norb, nelec[spin], p, q).toarray()
                if spin == 0:
                    ref = np.kron(Es, np.eye(db))
                else:
                    ref = np.kron(np.eye(da), Es)
                np.testing.assert_array_equal(M, ref.real)
