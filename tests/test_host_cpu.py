"""Host-side checks that need no GPU: the C-ABI library loads, exports every
declared entry point, and its host routines (string tables, Givens
decomposition) match the oracle / reconstruct their input."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import strings as ost
from paper_2605_03123_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2605_03123_amd", "libffx.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libffx.so not built")


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            names |= set(re.findall(r"^\s*(?:const\s+)?\w+\*?\s+\**(ffx_\w+)\s*\(", txt, re.M))
    return sorted(names)


def test_every_declared_symbol_is_exported():
    lib = ctypes.CDLL(LIB)
    names = _declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n


def test_string_tables_are_bit_exact():
    from paper_2605_03123_amd import ffx
    for norb, n in [(1, 0), (1, 1), (5, 2), (8, 4), (12, 6), (16, 8), (16, 3), (18, 9)]:
        np.testing.assert_array_equal(ffx.strings(norb, n), ost.strings(norb, n).astype(np.uint64))
        assert ffx.dim(norb, n) == ost.dim(norb, n)


def _reconstruct(p, c, s, ph, norb):
    M = np.eye(norb, dtype=complex)
    for pk, ck, sk in zip(p, c, s):
        G = np.eye(norb, dtype=complex)
        G[pk, pk], G[pk, pk + 1], G[pk + 1, pk], G[pk + 1, pk + 1] = ck, sk, -np.conj(sk), ck
        M = G @ M
    return np.diag(np.exp(1j * ph)) @ M


@pytest.mark.parametrize("norb", [1, 2, 3, 8, 16, 18])
def test_givens_decomposition_reconstructs(norb):
    from paper_2605_03123_amd import ffx
    r = synth.rng(norb)
    for U in (synth.random_unitary(r, norb), synth.random_orthogonal(r, norb).astype(complex),
              np.eye(norb, dtype=complex), np.diag(np.exp(1j * r.normal(size=norb)))):
        p, c, s, ph = ffx.givens_decomposition(U)
        assert len(p) == norb * (norb - 1) // 2
        assert np.all((p >= 0) & (p < max(norb - 1, 1)))
        np.testing.assert_allclose(_reconstruct(p, c, s, ph, norb), U, atol=1e-14)
        if np.all(U.imag == 0):
            assert np.all(s.imag == 0) and np.all(np.isin(ph, [0.0, np.pi]))


def test_errors_are_reported_not_raised():
    from paper_2605_03123_amd import ffx
    with pytest.raises(ffx.FFXError) as e:
        ffx.givens_decomposition(np.ones((3, 3)))
    assert e.value.code == -2
    with pytest.raises(ffx.FFXError) as e:
        ffx.givens_decomposition(np.full((2, 2), np.nan))
    assert e.value.code == -1
    with pytest.raises(ValueError):
        ffx.dim(33, 1)
    with pytest.raises(ValueError):
        ffx.dim(4, 5)
