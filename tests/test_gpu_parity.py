"""GPU parity: the HIP path (through the C ABI) against the oracle, element by element.

complex128: max |amplitude difference| <= 1e-12 with no phase alignment (every
gate here has exactly one correct result).  complex64: <= 1e-5 against the
oracle run on the upcast of the complex64-rounded inputs (the kernel's own
arithmetic error); for the rotation, the config-1 chain and the DF steps the
error against the oracle on the original complex128 input (which adds the input
rounding) is asserted to the same bound and recorded beside it.  Energies and
gradients: 1e-12 (complex128) / 1e-5 (complex64) relative to max(1, |reference|).
Every chain here, multi-step and symmetric product formulas included, is held to
these single-gate bounds.
"""
import numpy as np
import pytest
import torch

from oracle import gates as og
from oracle import hamiltonian as oh
from oracle import lucj as ol
from oracle import strings as ost
from paper_2605_03123_amd import synth
from errlog import AMP, REL, record

pytestmark = pytest.mark.gpu

TOL = {torch.complex128: AMP["complex128"], torch.complex64: AMP["complex64"]}
RTOL = {torch.complex128: REL["complex128"], torch.complex64: REL["complex64"]}
DTYPES = [torch.complex128, torch.complex64]


@pytest.fixture(scope="module")
def ffx():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_2605_03123_amd import ffx as mod
    return mod


def _dims(norb, nelec):
    return ost.dim(norb, nelec[0]), ost.dim(norb, nelec[1])


def _to_dev(vec, dtype):
    return torch.from_numpy(np.ascontiguousarray(vec)).to(dtype).to("cuda:0")


def _ref_input(t):
    """The oracle's input: the device state's own values (c64 inputs upcast exactly)."""
    return t.detach().cpu().to(torch.complex128).numpy()


def _maxdiff(t, ref):
    return float(np.max(np.abs(t.detach().cpu().to(torch.complex128).numpy() - ref))) if ref.size else 0.0


# sizes that span several 256-column tiles and leave ragged tails, edge sectors included
ROT_CASES = [
    (1, (0, 1)), (1, (1, 1)), (2, (1, 1)), (3, (0, 2)), (3, (3, 1)), (4, (2, 2)), (5, (2, 3)),
    (6, (3, 3)), (7, (3, 4)), (8, (4, 4)), (8, (1, 7)), (9, (4, 5)), (10, (5, 5)), (10, (3, 6)),
    (11, (5, 4)), (12, (6, 6)),
]


def test_plan_string_tables_bit_exact(ffx):
    for norb, nelec in [(8, (4, 3)), (12, (6, 6)), (16, (8, 8)), (1, (0, 1))]:
        p = ffx.get_plan(norb, nelec)
        for spin in (0, 1):
            np.testing.assert_array_equal(p.strings(spin), ost.strings(norb, nelec[spin]).astype(np.uint64))


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("norb,nelec", ROT_CASES)
def test_orbital_rotation(ffx, dtype, norb, nelec):
    r = synth.rng([norb, nelec[0], nelec[1]])
    da, db = _dims(norb, nelec)
    v0 = synth.random_state(r, da, db)
    vec = _to_dev(v0, dtype)
    x = _ref_input(vec)
    Ua, Ub = synth.random_unitary(r, norb), synth.random_unitary(r, norb)
    O = synth.random_orthogonal(r, norb)
    out = ffx.apply_orbital_rotation(vec, Ua, norb, nelec, U_b=Ub)
    err = record("orbital_rotation", dtype, "amplitude", _maxdiff(out, og.apply_orbital_rotation(x, Ua, norb, nelec, U_b=Ub)),
                 TOL[dtype], norb=norb, nelec=list(nelec))
    assert err <= TOL[dtype]
    if dtype == torch.complex64:
        err = record("orbital_rotation", dtype, "amplitude_vs_original_input",
                     _maxdiff(out, og.apply_orbital_rotation(v0, Ua, norb, nelec, U_b=Ub)), TOL[dtype], norb=norb,
                     nelec=list(nelec))
        assert err <= TOL[dtype]
    out = ffx.apply_orbital_rotation(vec, Ua, norb, nelec)
    assert _maxdiff(out, og.apply_orbital_rotation(x, Ua, norb, nelec)) <= TOL[dtype]
    out = ffx.apply_orbital_rotation(vec, O, norb, nelec)
    assert _maxdiff(out, og.apply_orbital_rotation(x, O, norb, nelec)) <= TOL[dtype]
    # input untouched by the functional form
    assert _maxdiff(vec, x) == 0.0


def test_orbital_rotation_in_place_and_identity(ffx):
    norb, nelec = 8, (4, 4)
    r = synth.rng(5)
    vec = _to_dev(synth.random_state(r, 70, 70), torch.complex128)
    x = _ref_input(vec)
    ffx.apply_orbital_rotation(vec, np.eye(norb), norb, nelec, out=vec)
    assert _maxdiff(vec, x) <= 1e-15
    D = np.diag(np.exp(1j * r.normal(size=norb)))
    out = ffx.apply_orbital_rotation(vec, D, norb, nelec)
    assert _maxdiff(out, og.apply_orbital_rotation(x, D, norb, nelec)) <= 1e-12


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("norb,nelec", [(3, (1, 2)), (8, (4, 4)), (10, (5, 4)), (12, (6, 6)), (17, (2, 3))])
def test_phase_gates(ffx, dtype, norb, nelec):
    r = synth.rng([7, norb])
    da, db = _dims(norb, nelec)
    vec = _to_dev(synth.random_state(r, da, db), dtype)
    x = _ref_input(vec)
    la, lb = r.normal(size=norb), r.normal(size=norb)
    out = ffx.apply_num_op_sum_evolution(vec, la, 0.7, norb, nelec, lam_b=lb)
    assert _maxdiff(out, og.apply_num_op_sum_evolution(x, la, 0.7, norb, nelec, lam_b=lb)) <= TOL[dtype]
    Jaa, Jab, Jbb = (synth.random_symmetric(r, norb, 1.0) for _ in range(3))
    out = ffx.apply_diag_coulomb_evolution(vec, Jaa, 0.3, norb, nelec, J_ab=Jab, J_bb=Jbb)
    ref = og.apply_diag_coulomb_evolution(x, Jaa, 0.3, norb, nelec, J_ab=Jab, J_bb=Jbb)
    assert record("diag_coulomb", dtype, "amplitude", _maxdiff(out, ref), TOL[dtype], norb=norb) <= TOL[dtype]
    out = ffx.apply_diag_coulomb_evolution(vec, Jaa, -1.3, norb, nelec)
    assert _maxdiff(out, og.apply_diag_coulomb_evolution(x, Jaa, -1.3, norb, nelec)) <= TOL[dtype]


@pytest.mark.parametrize("dtype", DTYPES)
def test_rotation_coulomb_workload(ffx, dtype):
    """norb=8 (4,4): U, exp(-1/2 i t sum J n n) with t=0.3, then U^dag on a random state (seed 0)."""
    w = synth.workload_rotation_coulomb(0)
    norb, nelec, d = w.norb, w.nelec, w.data
    vec = _to_dev(d["vec"], dtype)
    x = _ref_input(vec)
    out = ffx.apply_orbital_rotation(vec, d["U"], norb, nelec)
    ffx.apply_diag_coulomb_evolution(out, d["J"], d["t"], norb, nelec, out=out)
    ffx.apply_orbital_rotation(out, d["U"].conj().T, norb, nelec, out=out)

    def chain(v):
        ref = og.apply_orbital_rotation(v, d["U"], norb, nelec)
        ref = og.apply_diag_coulomb_evolution(ref, d["J"], d["t"], norb, nelec)
        return og.apply_orbital_rotation(ref, d["U"].conj().T, norb, nelec)

    ref = chain(x)
    assert record("config1_rotation_coulomb", dtype, "amplitude", _maxdiff(out, ref), TOL[dtype]) <= TOL[dtype]
    if dtype == torch.complex64:
        err = record("config1_rotation_coulomb", dtype, "amplitude_vs_original_input", _maxdiff(out, chain(d["vec"])),
                     TOL[dtype])
        assert err <= TOL[dtype]
    nrm = float(torch.linalg.vector_norm(out.to(torch.complex128)))
    assert abs(nrm - np.linalg.norm(ref)) <= TOL[dtype]


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("order,n_steps", [(0, 1), (0, 3), (1, 2), (2, 1)])
@pytest.mark.parametrize("norb,nelec,L", [(6, (3, 3), 3), (8, (4, 3), 4)])
def test_df_trotter(ffx, dtype, order, n_steps, norb, nelec, L):
    r = synth.rng([11, norb, order])
    ham = synth.df_hamiltonian(r, norb, L)
    da, db = _dims(norb, nelec)
    v0 = synth.random_state(r, da, db)
    vec = _to_dev(v0, dtype)
    x = _ref_input(vec)
    out = ffx.simulate_trotter_double_factorized(vec, ham, 0.1 * n_steps, norb, nelec, n_steps=n_steps, order=order)
    ref = oh.simulate_trotter(x, ham, 0.1 * n_steps, norb, nelec, n_steps=n_steps, order=order)
    tag = dict(norb=norb, nelec=list(nelec), L=L, order=order, n_steps=n_steps)
    assert record("df_trotter", dtype, "amplitude", _maxdiff(out, ref), TOL[dtype], **tag) <= TOL[dtype]
    if dtype == torch.complex64:
        ref0 = oh.simulate_trotter(v0, ham, 0.1 * n_steps, norb, nelec, n_steps=n_steps, order=order)
        err = record("df_trotter", dtype, "amplitude_vs_original_input", _maxdiff(out, ref0), TOL[dtype], **tag)
        assert err <= TOL[dtype]


def test_df_trotter_complex_basis(ffx):
    r = synth.rng(12)
    norb, nelec = 7, (3, 4)
    ham = synth.df_hamiltonian(r, norb, 3)
    ham.U = np.array([synth.random_unitary(r, norb) for _ in range(3)])
    vec = _to_dev(synth.random_state(r, 35, 35), torch.complex128)
    x = _ref_input(vec)
    out = ffx.simulate_trotter_double_factorized(vec, ham, 0.2, norb, nelec, n_steps=2, order=0)
    assert _maxdiff(out, oh.simulate_trotter(x, ham, 0.2, norb, nelec, n_steps=2, order=0)) <= 1e-12


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("norb,nelec,n_reps", [(4, (2, 1), 2), (6, (3, 3), 3), (8, (4, 4), 2), (9, (3, 4), 1)])
def test_lucj_forward(ffx, dtype, norb, nelec, n_reps):
    params = synth.lucj_params(synth.rng([13, norb]), norb, n_reps, scale=0.3)
    out = ffx.apply_lucj(params, norb, nelec, n_reps, dtype=dtype)
    err = _maxdiff(out, ol.apply_lucj(params, norb, nelec, n_reps))
    assert record("lucj_forward", dtype, "amplitude", err, TOL[dtype], norb=norb, n_reps=n_reps) <= TOL[dtype]


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("norb,nelec", [(4, (2, 2)), (8, (4, 4)), (9, (5, 3))])
def test_df_energy(ffx, dtype, norb, nelec):
    r = synth.rng([14, norb])
    ham = synth.df_hamiltonian(r, norb, norb)
    da, db = _dims(norb, nelec)
    vec = _to_dev(synth.random_state(r, da, db), dtype)
    x = _ref_input(vec)
    e = ffx.df_energy(vec, ham, norb, nelec)
    ref = oh.df_energy(x, ham, norb, nelec)
    err = abs(e - ref.real) / max(1.0, abs(ref.real))
    assert record("df_energy", dtype, "energy_rel", err, RTOL[dtype], norb=norb) <= RTOL[dtype]
    assert ffx.df_energy(vec, ham, norb, nelec) == e   # fixed reduction order


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("norb,nelec,n_reps", [(4, (2, 1), 2), (6, (3, 3), 2), (8, (4, 4), 1), (5, (0, 2), 1),
                                             (5, (5, 3), 1), (7, (1, 6), 2)])
def test_lucj_energy_grad_matches_oracle_adjoint(ffx, dtype, norb, nelec, n_reps):
    r = synth.rng([15, norb])
    params = synth.lucj_params(r, norb, n_reps, scale=0.3)
    ham = synth.df_hamiltonian(r, norb, 2)
    e, g = ffx.lucj_energy_grad(params, ham, norb, nelec, n_reps, dtype=dtype)
    eo, go = ol.grad_adjoint(params, ham, norb, nelec, n_reps)
    tol = RTOL[dtype]
    tag = dict(norb=norb, nelec=list(nelec), n_reps=n_reps)
    assert record("lucj_energy", dtype, "energy_rel", abs(e - eo) / max(1, abs(eo)), tol, **tag) <= tol
    err = np.max(np.abs(g - go)) / max(1, np.max(np.abs(go)))
    assert record("lucj_gradient_vs_oracle_adjoint", dtype, "grad_rel", err, tol, **tag) <= tol


@pytest.mark.parametrize("mode", ["auto", "rot"])
@pytest.mark.parametrize("nx,ny", [(4, 2), (4, 3)])
def test_lucj_energy_grad_hubbard(ffx, monkeypatch, mode, nx, ny):
    """LUCJ under the Hubbard model: the costate's one-body term from the sparse excitation tables (auto)
    or through the eigenbasis of h (rot), against the oracle's adjoint gradient."""
    if mode != "auto":
        monkeypatch.setenv("FFX_ONEBODY", mode)
    norb, nelec = nx * ny, synth.hubbard_filling(nx, ny)
    ham = synth.hubbard_2d(nx, ny)
    params = synth.lucj_params(synth.rng([16, nx, ny]), norb, 2, scale=0.3)
    e, g = ffx.lucj_energy_grad(params, ham, norb, nelec, 2)
    eo, go = ol.grad_adjoint(params, ham, norb, nelec, 2)
    tol = RTOL[torch.complex128]
    assert abs(e - eo) <= tol * max(1, abs(eo))
    err = np.max(np.abs(g - go)) / max(1, np.max(np.abs(go)))
    assert record("lucj_gradient_hubbard_" + mode, torch.complex128, "grad_rel", err, tol, lattice=[nx, ny]) <= tol


def test_lucj_gradient_matches_central_differences_on_gpu(ffx):
    norb, nelec, n_reps = 8, (4, 4), 2
    r = synth.rng(16)
    params = synth.lucj_params(r, norb, n_reps)
    ham = synth.df_hamiltonian(r, norb, norb)
    e, g = ffx.lucj_energy_grad(params, ham, norb, nelec, n_reps)
    idx = synth.fd_indices(len(params), 10)
    h = 1e-5
    for j in idx:
        d = np.zeros_like(params)
        d[j] = h
        ep = ffx.lucj_energy_grad(params + d, ham, norb, nelec, n_reps)[0]
        em = ffx.lucj_energy_grad(params - d, ham, norb, nelec, n_reps)[0]
        assert abs((ep - em) / (2 * h) - g[j]) <= 1e-7 * max(1, np.max(np.abs(g)))


def test_autograd_function(ffx):
    norb, nelec, n_reps = 4, (2, 2), 1
    r = synth.rng(17)
    p = torch.tensor(synth.lucj_params(r, norb, n_reps, scale=0.3), requires_grad=True)
    ham = synth.df_hamiltonian(r, norb, 2)
    E = ffx.LUCJEnergy.apply(p, ham, norb, nelec, n_reps)
    E.backward()
    _, go = ol.grad_adjoint(p.detach().numpy(), ham, norb, nelec, n_reps)
    np.testing.assert_allclose(p.grad.numpy(), go, atol=RTOL[torch.complex128] * max(1.0, np.max(np.abs(go))))


def test_errors_do_not_crash(ffx):
    vec = torch.zeros((6, 6), dtype=torch.complex128, device="cuda:0")
    with pytest.raises(ffx.FFXError):
        ffx.apply_orbital_rotation(vec, np.ones((4, 4)), 4, (2, 2))
    with pytest.raises(ValueError):
        ffx.apply_orbital_rotation(vec, np.eye(4), 4, (2, 1))
    with pytest.raises(TypeError):
        ffx.apply_orbital_rotation(vec.to(torch.complex64), np.eye(4), 4, (2, 2), out=vec)


@pytest.fixture(scope="module")
def small_segment_plans(ffx):
    """Plans whose segments are forced to be tiny, so that rotations cross segments
    and run through whole-spin window passes between segment passes: one
    segment per run of configurations sharing the orbitals above the window
    (FFX_SEG_PACK=0), with the rotation on the pair straddling the window
    applied at load (FFX_CROSS_AT_LOAD=1) or, as by default when several pairs
    cross, left to the window passes; and runs packed back to back (that
    rotation takes a window pass)."""
    import os
    plans = {}
    old = {k: os.environ.get(k) for k in ("FFX_SEG_MAX", "FFX_SEG_PACK", "FFX_CROSS_AT_LOAD")}
    os.environ["FFX_SEG_MAX"] = "24"
    try:
        for pack, at_load in (("0", "1"), ("0", None), ("1", None)):
            os.environ["FFX_SEG_PACK"] = pack
            if at_load:
                os.environ["FFX_CROSS_AT_LOAD"] = at_load
            else:
                os.environ.pop("FFX_CROSS_AT_LOAD", None)
            for norb, nelec, dt in [(8, (4, 4), torch.complex128), (10, (3, 6), torch.complex128),
                                    (9, (4, 5), torch.complex64), (11, (5, 4), torch.complex128)]:
                plans[(norb, nelec, dt, pack, at_load)] = ffx.Plan(norb, nelec, dt)
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    return plans


def test_segmented_paths(ffx, small_segment_plans):
    for (norb, nelec, dtype, _, _), plan in small_segment_plans.items():
        r = synth.rng([21, norb])
        da, db = _dims(norb, nelec)
        vec = _to_dev(synth.random_state(r, da, db), dtype)
        x = _ref_input(vec)
        U = synth.random_unitary(r, norb)
        out = ffx.apply_orbital_rotation(vec, U, norb, nelec, plan=plan)
        assert _maxdiff(out, og.apply_orbital_rotation(x, U, norb, nelec)) <= TOL[dtype]
        ham = synth.df_hamiltonian(r, norb, 3)
        out = ffx.simulate_trotter_double_factorized(vec, ham, 0.2, norb, nelec, n_steps=2, order=1, plan=plan)
        ref = oh.simulate_trotter(x, ham, 0.2, norb, nelec, n_steps=2, order=1)
        err = record("segmented_df_trotter_s1", dtype, "amplitude", _maxdiff(out, ref), TOL[dtype], norb=norb)
        assert err <= TOL[dtype]
        e = ffx.df_energy(vec, ham, norb, nelec, plan=plan)
        ref = oh.df_energy(x, ham, norb, nelec).real
        assert abs(e - ref) <= RTOL[dtype] * max(1, abs(ref))
        params = synth.lucj_params(r, norb, 2, scale=0.3)
        out = ffx.apply_lucj(params, norb, nelec, 2, dtype=dtype, plan=plan)
        assert _maxdiff(out, ol.apply_lucj(params, norb, nelec, 2)) <= TOL[dtype]


def test_segmented_paths_in_place_and_gradients(ffx, small_segment_plans):
    # crossing rotations move the state between the working buffers; in-place
    # calls must still end in the caller's buffer, and the adjoint gradient runs
    # programs that end in accumulation or in a reduction only
    for (norb, nelec, dtype, _, _), plan in small_segment_plans.items():
        r = synth.rng([22, norb])
        da, db = _dims(norb, nelec)
        vec = _to_dev(synth.random_state(r, da, db), dtype)
        x = _ref_input(vec)
        ref = x
        for k in range(3):
            U = synth.random_unitary(r, norb)
            ffx.apply_orbital_rotation(vec, U, norb, nelec, out=vec, plan=plan)
            ref = og.apply_orbital_rotation(ref, U, norb, nelec)
            assert _maxdiff(vec, ref) <= TOL[dtype]
        ham = synth.df_hamiltonian(r, norb, 2)
        ffx.simulate_trotter_double_factorized(vec, ham, 0.1, norb, nelec, n_steps=1, order=0, out=vec, plan=plan)
        ref = oh.simulate_trotter(ref, ham, 0.1, norb, nelec, n_steps=1, order=0)
        err = record("segmented_in_place_chain", dtype, "amplitude", _maxdiff(vec, ref), TOL[dtype], norb=norb)
        assert err <= TOL[dtype]
        params = synth.lucj_params(r, norb, 2, scale=0.3)
        e, g = ffx.lucj_energy_grad(params, ham, norb, nelec, 2, dtype=dtype, plan=plan)
        eo, go = ol.grad_adjoint(params, ham, norb, nelec, 2)
        tol = RTOL[dtype]
        assert abs(e - float(np.real(eo))) <= tol * max(1.0, abs(float(np.real(eo))))
        assert np.max(np.abs(g - go)) <= tol * max(1.0, np.max(np.abs(go)))


def test_lucj_energy_grad_returns_the_ansatz_state(ffx):
    # psi_out receives psi(theta) even though the reverse sweep uncomputes its own copy
    norb, nelec, n_reps = 6, (3, 3), 2
    w = synth.workload_lucj(norb, n_reps, 3, seed=12, nelec=nelec)
    plan = ffx.get_plan(norb, nelec, torch.complex128, 0)
    out = torch.zeros((plan.dim_a, plan.dim_b), dtype=torch.complex128, device="cuda:0")
    ffx.lucj_energy_grad(w.data["params"], w.data["ham"], norb, nelec, n_reps, psi_out=out)
    assert _maxdiff(out, ol.apply_lucj(w.data["params"], norb, nelec, n_reps)) <= 1e-12


def test_lucj_gradient_row_pair_transition_path(ffx):
    # the transition one-body matrices from row pairs (the path above 16
    # orbitals), forced at small sizes, against the oracle's adjoint gradient
    import os
    norb, nelec, n_reps = 7, (3, 4), 2
    r = synth.rng(23)
    params = synth.lucj_params(r, norb, n_reps, scale=0.3)
    ham = synth.df_hamiltonian(r, norb, 3)
    eo, go = ol.grad_adjoint(params, ham, norb, nelec, n_reps)
    os.environ["FFX_RDM_PAIRS"] = "1"
    try:
        plans = {dt: ffx.Plan(norb, nelec, dt) for dt in (torch.complex128, torch.complex64)}
    finally:
        del os.environ["FFX_RDM_PAIRS"]
    for dt, plan in plans.items():
        e, g = ffx.lucj_energy_grad(params, ham, norb, nelec, n_reps, dtype=dt, plan=plan)
        tol = RTOL[dt]
        assert abs(e - float(np.real(eo))) <= tol * max(1.0, abs(float(np.real(eo))))
        assert np.max(np.abs(g - go)) <= tol * max(1.0, np.max(np.abs(go)))



@pytest.fixture(scope="module")
def plane_plans(ffx):
    """complex128 plans whose all-real visits hold rows as two planes (real parts, imaginary parts) even
    where whole rows fit in LDS (FFX_PLANES_ALL), in both block sizes of the plane pass."""
    import os
    plans = {}
    old = {k: os.environ.get(k) for k in ("FFX_PLANES_ALL", "FFX_PLANES")}
    os.environ["FFX_PLANES_ALL"] = "1"
    try:
        for threads in ("512", "768"):
            os.environ["FFX_PLANES"] = threads
            for norb, nelec in [(6, (3, 3)), (8, (4, 3)), (9, (4, 5)), (10, (5, 5))]:
                plans[(norb, nelec, threads)] = ffx.Plan(norb, nelec, torch.complex128)
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    return plans


def test_plane_passes_against_oracle(ffx, plane_plans):
    """Real rotations on row planes: DF steps (S_0, S_1, two steps; real U_t, the one-body factor making the
    first rotation complex), the DF energy (reductions), the Hamiltonian action (accumulation), LUCJ energy and
    gradient, and a real orbital rotation in place, against the oracle."""
    _check_plane_plans(ffx, plane_plans, 24)


@pytest.fixture(scope="module")
def plane_segment_plans(ffx):
    """complex128 plans whose plane passes hold rows split into segments (FFX_PLANE_SEG_MAX caps a plane
    segment at a few dozen amplitudes), as rows longer than the plane kernel's capacity are at 18 orbitals:
    the rotations on the orbitals above the plane window run as whole-spin window passes between plane
    passes."""
    import os
    plans = {}
    old = {k: os.environ.get(k) for k in ("FFX_PLANES_ALL", "FFX_PLANE_SEG_MAX")}
    os.environ["FFX_PLANES_ALL"] = "1"
    try:
        for cap in ("24", "40"):
            os.environ["FFX_PLANE_SEG_MAX"] = cap
            for norb, nelec in [(8, (4, 4)), (9, (4, 5)), (10, (5, 5)), (11, (5, 4))]:
                plans[(norb, nelec, cap)] = ffx.Plan(norb, nelec, torch.complex128)
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    return plans


def test_plane_segment_passes_against_oracle(ffx, plane_segment_plans):
    """The same checks on plane passes over row segments, with window passes between them."""
    _check_plane_plans(ffx, plane_segment_plans, 25)


def _check_plane_plans(ffx, plans, seed):
    for (norb, nelec, threads), plan in plans.items():
        print(f"plane passes norb={norb} nelec={nelec} variant={threads}", flush=True)
        r = synth.rng([seed, norb, int(threads)])
        da, db = _dims(norb, nelec)
        vec = _to_dev(synth.random_state(r, da, db), torch.complex128)
        x = _ref_input(vec)
        ham = synth.df_hamiltonian(r, norb, 3)
        for order, n in ((0, 2), (1, 1)):
            out = ffx.simulate_trotter_double_factorized(vec, ham, 0.1 * n, norb, nelec, n_steps=n, order=order,
                                                         plan=plan)
            ref = oh.simulate_trotter(x, ham, 0.1 * n, norb, nelec, n_steps=n, order=order)
            err = record("plane_df_trotter", torch.complex128, "amplitude", _maxdiff(out, ref), 1e-12, norb=norb,
                         threads=int(threads))
            assert err <= 1e-12
        e = ffx.df_energy(vec, ham, norb, nelec, plan=plan)
        ref = oh.df_energy(x, ham, norb, nelec).real
        assert abs(e - ref) <= 1e-12 * max(1.0, abs(ref))
        hv = ffx.apply_df_hamiltonian(vec, ham, norb, nelec, plan=plan)
        ref = oh.apply_df_hamiltonian(x, ham, norb, nelec)
        assert _maxdiff(hv, ref) <= 1e-12 * max(1.0, float(np.abs(ref).max()))
        O = synth.random_orthogonal(r, norb)
        v2 = vec.clone()
        ffx.apply_orbital_rotation(v2, O, norb, nelec, out=v2, plan=plan)
        assert _maxdiff(v2, og.apply_orbital_rotation(x, O, norb, nelec)) <= 1e-12
        params = synth.lucj_params(r, norb, 2, scale=0.3)
        e, g = ffx.lucj_energy_grad(params, ham, norb, nelec, 2, plan=plan)
        eo, go = ol.grad_adjoint(params, ham, norb, nelec, 2)
        assert abs(e - float(np.real(eo))) <= 1e-12 * max(1.0, abs(float(np.real(eo))))
        assert np.max(np.abs(g - go)) <= 1e-12 * max(1.0, np.max(np.abs(go)))


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("switch", ["scatter", "gather", "transpose"])
def test_layout_switch_variants(ffx, monkeypatch, switch, dtype):
    """Every way a program switches layout between the visits of the two spins: the pass before the switch
    stores its rows as columns of the new layout (scatter), the pass after it gathers them (gather), or a
    transpose runs in between; square and rectangular states, whole rows and forced small segments (whose
    crossing rotations take window passes), in both precisions, for a DF step (S_1, two steps), the DF
    energy (reductions only), the Hamiltonian action (accumulation) and the LUCJ energy and gradient."""
    monkeypatch.setenv("FFX_SCATTER", "1" if switch == "scatter" else "0")
    monkeypatch.setenv("FFX_GATHER", "1" if switch == "gather" else "0")
    import os
    cases = [(8, (4, 4), None), (9, (3, 5), None), (10, (3, 6), "24")]
    for norb, nelec, seg_max in cases:
        print(f"layout switch {switch} {dtype} norb={norb} nelec={nelec} seg_max={seg_max}", flush=True)
        if seg_max:
            os.environ["FFX_SEG_MAX"] = seg_max
            try:
                plan = ffx.Plan(norb, nelec, dtype)
            finally:
                del os.environ["FFX_SEG_MAX"]
        else:
            plan = ffx.Plan(norb, nelec, dtype)
        r = synth.rng([26, norb, len(switch)])
        da, db = _dims(norb, nelec)
        vec = _to_dev(synth.random_state(r, da, db), dtype)
        x = _ref_input(vec)
        ham = synth.df_hamiltonian(r, norb, 3)
        out = ffx.simulate_trotter_double_factorized(vec, ham, 0.2, norb, nelec, n_steps=2, order=1, plan=plan)
        ref = oh.simulate_trotter(x, ham, 0.2, norb, nelec, n_steps=2, order=1)
        assert _maxdiff(out, ref) <= TOL[dtype]
        e = ffx.df_energy(vec, ham, norb, nelec, plan=plan)
        ref = oh.df_energy(x, ham, norb, nelec).real
        assert abs(e - ref) <= RTOL[dtype] * max(1.0, abs(ref))
        hv = ffx.apply_df_hamiltonian(vec, ham, norb, nelec, plan=plan)
        ref = oh.apply_df_hamiltonian(x, ham, norb, nelec)
        assert _maxdiff(hv, ref) <= RTOL[dtype] * max(1.0, float(np.abs(ref).max()))
        params = synth.lucj_params(r, norb, 2, scale=0.3)
        e, g = ffx.lucj_energy_grad(params, ham, norb, nelec, 2, dtype=dtype, plan=plan)
        eo, go = ol.grad_adjoint(params, ham, norb, nelec, 2)
        assert abs(e - float(np.real(eo))) <= RTOL[dtype] * max(1.0, abs(float(np.real(eo))))
        assert np.max(np.abs(g - go)) <= RTOL[dtype] * max(1.0, np.max(np.abs(go)))
