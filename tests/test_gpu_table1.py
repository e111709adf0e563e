"""GPU parity of the remaining Table 1 gates, the Slater-determinant state and the UCJ forward pass
through the C ABI, against the oracle (complex128 <= 1e-12, complex64 <= 1e-5 per amplitude)."""
import numpy as np
import pytest
import torch

from oracle import gates as og
from oracle import strings as ost
from paper_2605_03123_amd import synth

pytestmark = pytest.mark.gpu

TOL = {torch.complex128: 1e-12, torch.complex64: 1e-5}
DTYPES = [torch.complex128, torch.complex64]
# sizes the oracle's compound matrices finish in seconds, one above 16 orbitals, a full spin
CASES = [(4, (2, 2)), (7, (3, 4)), (9, (5, 3)), (12, (6, 5)), (20, (3, 2)), (5, (0, 5))]


@pytest.fixture(scope="module")
def ffx():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_2605_03123_amd import ffx as mod
    return mod


def _dims(norb, nelec):
    return ost.dim(norb, nelec[0]), ost.dim(norb, nelec[1])


def _to_dev(vec, dtype):
    return torch.from_numpy(np.ascontiguousarray(vec)).to(dtype).to("cuda:0")


def _host(t):
    return t.detach().cpu().to(torch.complex128).numpy()


def _maxdiff(t, ref):
    return float(np.max(np.abs(_host(t) - ref))) if ref.size else 0.0


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("norb,nelec", CASES)
def test_table1_gates(ffx, dtype, norb, nelec):
    print(f"Table 1 gates norb={norb} nelec={nelec} {dtype}", flush=True)
    r = synth.rng([61, norb, *nelec])
    vec = _to_dev(synth.random_state(r, *_dims(norb, nelec)), dtype)
    x = _host(vec)
    p, q = 0, norb - 1
    cases = [
        (lambda: ffx.apply_num_interaction(vec, 0.8, p, 0, norb, nelec),
         lambda: og.apply_num_interaction(x, 0.8, p, 0, norb, nelec)),
        (lambda: ffx.apply_num_interaction(vec, -0.3, q, 1, norb, nelec),
         lambda: og.apply_num_interaction(x, -0.3, q, 1, norb, nelec)),
        (lambda: ffx.apply_num_num_interaction(vec, 1.1, p, 0, q, 1, norb, nelec),
         lambda: og.apply_num_num_interaction(x, 1.1, p, 0, q, 1, norb, nelec)),
        (lambda: ffx.apply_num_num_interaction(vec, 0.6, q, 1, p, 0, norb, nelec),
         lambda: og.apply_num_num_interaction(x, 0.6, q, 1, p, 0, norb, nelec)),
        (lambda: ffx.apply_num_num_interaction(vec, -0.9, q, 1, q, 1, norb, nelec),
         lambda: og.apply_num_num_interaction(x, -0.9, q, 1, q, 1, norb, nelec)),
    ]
    if norb > 1:
        cases += [
            (lambda: ffx.apply_num_num_interaction(vec, 0.5, 1, 0, p, 0, norb, nelec),
             lambda: og.apply_num_num_interaction(x, 0.5, 1, 0, p, 0, norb, nelec)),
            (lambda: ffx.apply_givens_rotation(vec, 0.7, p, q, 0, norb, nelec),
             lambda: og.apply_givens_rotation(x, 0.7, p, q, 0, norb, nelec)),
            (lambda: ffx.apply_givens_rotation(vec, -1.2, 1, 0, 1, norb, nelec),
             lambda: og.apply_givens_rotation(x, -1.2, 1, 0, 1, norb, nelec)),
            (lambda: ffx.apply_tunneling_interaction(vec, 0.45, q, p, 1, norb, nelec),
             lambda: og.apply_tunneling_interaction(x, 0.45, q, p, 1, norb, nelec)),
        ]
    Ma, Mb = synth.random_hermitian(r, norb, 0.5), synth.random_hermitian(r, norb, 0.5)
    cases.append((lambda: ffx.apply_quad_ham_evolution(vec, Ma, 0.8, norb, nelec, M_b=Mb),
                  lambda: og.apply_quad_ham_evolution(x, Ma, 0.8, norb, nelec, M_b=Mb)))
    for k, (gpu, ref) in enumerate(cases):
        assert _maxdiff(gpu(), ref()) <= TOL[dtype], k
    assert _maxdiff(vec, x) == 0.0


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("norb,nelec", [(4, (2, 2)), (9, (5, 3)), (12, (6, 6)), (5, (0, 5))])
def test_slater_determinant(ffx, dtype, norb, nelec):
    r = synth.rng([62, norb])
    Ua, Ub = synth.random_unitary(r, norb), synth.random_unitary(r, norb)
    occ_a = list(r.permutation(norb)[:nelec[0]])
    occ_b = list(r.permutation(norb)[:nelec[1]])
    out = ffx.slater_determinant(norb, nelec, occ_a=occ_a, occ_b=occ_b, U=Ua, U_b=Ub, dtype=dtype)
    assert _maxdiff(out, og.slater_determinant(norb, nelec, occ_a, occ_b, Ua, Ub)) <= TOL[dtype]
    out = ffx.slater_determinant(norb, nelec, dtype=dtype)  # Hartree-Fock
    assert _maxdiff(out, og.slater_determinant(norb, nelec)) == 0.0


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("norb,nelec,R,final", [(6, (3, 2), 2, True), (10, (5, 5), 3, False),
                                                (12, (6, 5), 1, True), (7, (1, 6), 2, True)])
def test_ucj_per_spin_full_j(ffx, dtype, norb, nelec, R, final):
    print(f"UCJ norb={norb} nelec={nelec} R={R} {dtype}", flush=True)
    r = synth.rng([63, norb, R])
    Ua = [synth.random_unitary(r, norb) for _ in range(R)]
    Ub = [synth.random_unitary(r, norb) for _ in range(R)]
    Jaa = [synth.random_symmetric(r, norb, 0.3) for _ in range(R)]
    Jbb = [synth.random_symmetric(r, norb, 0.3) for _ in range(R)]
    Jab = [r.normal(0.0, 0.3, (norb, norb)) for _ in range(R)]
    Fa = synth.random_unitary(r, norb) if final else None
    Fb = synth.random_unitary(r, norb) if final else None
    out = ffx.apply_ucj(norb, nelec, np.array(Ua), np.array(Jaa), U_b=np.array(Ub), J_ab=np.array(Jab),
                        J_bb=np.array(Jbb), final=Fa, final_b=Fb, dtype=dtype)
    ref = og.apply_ucj(norb, nelec, Ua, Jaa, U_b=Ub, J_ab=Jab, J_bb=Jbb, final_a=Fa, final_b=Fb)
    assert _maxdiff(out, ref) <= TOL[dtype]


def test_table1_argument_errors(ffx):
    norb, nelec = 4, (2, 2)
    vec = _to_dev(synth.random_state(synth.rng(64), *_dims(norb, nelec)), torch.complex128)
    for bad in (lambda: ffx.apply_num_interaction(vec, 0.1, 4, 0, norb, nelec),
                lambda: ffx.apply_num_interaction(vec, 0.1, 0, 2, norb, nelec),
                lambda: ffx.apply_givens_rotation(vec, 0.1, 1, 1, 0, norb, nelec),
                lambda: ffx.apply_tunneling_interaction(vec, float("inf"), 0, 1, 0, norb, nelec),
                lambda: ffx.apply_quad_ham_evolution(vec, np.triu(np.ones((4, 4))), 0.1, norb, nelec),
                lambda: ffx.slater_determinant(norb, nelec, occ_a=[1, 1]),
                lambda: ffx.slater_determinant(norb, nelec, occ_a=[0, 5])):
        with pytest.raises(ffx.FFXError):
            bad()


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("norb,nelec", [(6, (3, 2)), (10, (5, 5)), (20, (3, 2))])
def test_diagonal_gates_in_a_rotated_basis(ffx, dtype, norb, nelec):
    r = synth.rng([65, norb, *nelec])
    vec = _to_dev(synth.random_state(r, *_dims(norb, nelec)), dtype)
    x = _host(vec)
    B = synth.random_unitary(r, norb)
    lam, lam_b = r.normal(0, 1, norb), r.normal(0, 1, norb)
    out = ffx.apply_num_op_sum_evolution(vec, lam, 0.4, norb, nelec, lam_b=lam_b, orbital_rotation=B)
    ref = og.apply_in_basis(x, B, lambda v: og.apply_num_op_sum_evolution(v, lam, 0.4, norb, nelec, lam_b=lam_b),
                            norb, nelec)
    assert _maxdiff(out, ref) <= TOL[dtype]
    J, Jab = synth.random_symmetric(r, norb, 0.5), synth.random_symmetric(r, norb, 0.5)
    out = ffx.apply_diag_coulomb_evolution(vec, J, 0.4, norb, nelec, J_ab=Jab, orbital_rotation=B)
    ref = og.apply_in_basis(x, B, lambda v: og.apply_diag_coulomb_evolution(v, J, 0.4, norb, nelec, J_ab=Jab),
                            norb, nelec)
    assert _maxdiff(out, ref) <= TOL[dtype]


@pytest.mark.parametrize("dtype", DTYPES)
def test_large_orbital_counts(ffx, dtype):
    """UCJ, Slater state and quadratic-Hamiltonian evolution above 16 orbitals (three and four mask bytes)."""
    r = synth.rng(66)
    norb, nelec = 20, (3, 2)
    Ua, Ub = synth.random_unitary(r, norb), synth.random_unitary(r, norb)
    J = synth.random_symmetric(r, norb, 0.3)
    out = ffx.apply_ucj(norb, nelec, Ua[None], J[None], U_b=Ub[None], dtype=dtype)
    assert _maxdiff(out, og.apply_ucj(norb, nelec, [Ua], [J], U_b=[Ub])) <= TOL[dtype]
    norb, nelec = 32, (2, 2)
    U = synth.random_unitary(r, norb)
    out = ffx.slater_determinant(norb, nelec, occ_a=[31, 5], occ_b=[0, 16], U=U, dtype=dtype)
    assert _maxdiff(out, og.slater_determinant(norb, nelec, [31, 5], [0, 16], U)) <= TOL[dtype]
    norb, nelec = 24, (2, 1)
    vec = _to_dev(synth.random_state(r, *_dims(norb, nelec)), dtype)
    M = synth.random_hermitian(r, norb, 0.5)
    out = ffx.apply_quad_ham_evolution(vec, M, 0.7, norb, nelec)
    assert _maxdiff(out, og.apply_quad_ham_evolution(_host(vec), M, 0.7, norb, nelec)) <= TOL[dtype]
