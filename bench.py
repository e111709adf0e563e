"""Benchmark: seconds per double-factorized Trotter step at norb = 16, (8, 8).

    python bench.py [--steps K] [--warmup W] [--dtype c128|c64] [--no-cpu-baseline] [--no-lucj]
                    [--copy-calibration]

Workload: one first-order (S_0) Trotter step, dt = 0.1, of a DF Hamiltonian
with L = 16 terms (h ~ sym N(0, 0.5); U_t real orthogonal from QR; J_t ~ sym
N(0, 0.1)) on a random normalized 12870 x 12870 state, seed 0.  The state is
resident in HBM before timing; W untimed steps, then K timed steps bracketed by
device synchronization, timed with HIP events on the working stream (one per
step boundary: the mean is `value`, the median and interquartile range of the
single steps are reported beside it).  `value`
is the time per step in the primary precision (--dtype, complex128 by
default); the other precision is timed the same way and reported beside it.

Also reported (unless --no-batched): the batched energies + adjoint gradients
of 256 small sectors (norb 8-12) in both precisions.

Also reported (unless --no-hubbard): the Trotter-error workload of Sec. 6.2 on
the 2D Hubbard model (t = 1, U = 8, 4 x 8 lattice periodic in x, 1/8 filling,
T = 1): one Hamiltonian action, the exact evolution, Trotter runs of orders 1
and 2 and their errors, and beside it the same measurement on a 4 x 4 lattice
on the GPU (the cpu_baseline object holds the oracle's time for that one).

Also reported (unless --no-n18): one S_0 step at norb = 18, (9, 9), L = 18
(37.8 GB complex128) in both precisions with the HBM rate of each kernel family.

Also reported (unless --no-table1): the time per call of the other Table 1
gates, the Slater-determinant state, a 3-repetition UCJ forward pass and the
sampling of 1e5 configurations from the state and from a Slater determinant
(host uniforms in, host results out) at norb = 16, (8, 8), complex128.

Also reported (unless --no-lucj): the energy after one DF step under a second
DF Hamiltonian and its adjoint gradient in (h, J_t, U_t), and the LUCJ energy + adjoint gradient at
norb = 16, n_reps = 3, L = 16 in both precisions, and against it the
forward-only central finite-difference gradient (h = 1e-5) on 20 parameters
in complex128: its time, the extrapolated time for all parameters, and the
largest difference to the adjoint gradient.

Prints ONE JSON line with the metric, a roofline object for the dominant
kernel (the segment pass; per-launch durations measured live with HIP events
on the launch stream) and the oracle timed on a bounded sample of the same
step.  The roofline's `traffic` is the HBM byte count per launch from the
committed rocprofv3 FETCH_SIZE / WRITE_SIZE passes, used only while the
kernel sources still hash to the value recorded with them (else null).

--hubbard-only runs the Trotter-error leg alone (for profiling).

--copy-calibration adds device copies of a known size (for scaling the
FETCH_SIZE / WRITE_SIZE counters under rocprofv3) and skips the rest.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
NORB, NELEC, L, DT = 16, (8, 8), 16, 0.1
LUCJ_REPS, FD_H = 3, 1e-5
KERNEL_SOURCES = ("segpass.hip", "dev_common.h", "device.h")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_seg_pass_df_trotter_n16.txt")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2605_03123_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def committed_traffic(dtype_name: str):
    """HBM bytes per segment-pass launch from the committed counter passes, if still valid."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    with open(TRAFFIC_FILE) as fh:
        for line in fh:
            if "=" in line and not line.lstrip().startswith("#"):
                k, v = line.split("=", 1)
                kv[k.strip()] = v.strip()
    key = f"bytes_per_launch_{dtype_name}"
    if kv.get("kernel_sources_sha256") != kernel_source_hash() or key not in kv:
        return None
    return float(kv[key])


def cpu_baseline(ham, vec: np.ndarray, synth=None, hubbard_small=None) -> dict:
    """Time the oracle on a bounded sample of one Trotter step and scale to a whole step.

    The oracle applies each orbital rotation as Gamma' = C(U) Gamma C(U)^T with the compound matrix C(U)
    built from all dim^2 minors (float64 determinants for a real U, its rows spread over the host cores), and
    each diagonal Coulomb phase over the whole state.  Sample: R_c rows of C(U) for the first term's real
    U_t^dag, the products of R_g rows of C(U) with the real and the imaginary part of Gamma (the oracle's
    products for a real U), and one full diagonal-Coulomb phase.  Scaled: per rotation
    dim/R_c * t_C + 2 dim/R_g * t_G; per step (2L + 1) rotations and L phases (the oracle does not merge
    rotations; the step's one complex rotation, about twice the cost of a real one, is counted as real).
    Beside it: the wall time of a whole oracle step measured once, stored with the oracle's result for the
    16-orbital step (tests/golden/df_trotter_n16.txt).
    """
    from oracle import gates as og
    from oracle import strings as ost
    cores = len(os.sched_getaffinity(0))
    try:
        from threadpoolctl import threadpool_info
        blas_threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        blas_threads = cores
    workers = min(cores, 16)
    og.set_workers(workers)
    d = ost.dim(NORB, NELEC[0])
    U = np.asarray(ham.U[0]).conj().T
    R_c, R_g = 1024, 768
    t0 = time.perf_counter()
    rows = og.compound_matrix(U, NELEC[0], rows=np.arange(R_c))
    t_c = time.perf_counter() - t0
    og.set_workers(1)
    A = np.ascontiguousarray(rows[:R_g])
    re, im = np.ascontiguousarray(vec.real), np.ascontiguousarray(vec.imag)
    t0 = time.perf_counter()
    _ = A @ re
    _ = A @ im
    t_g = time.perf_counter() - t0
    t0 = time.perf_counter()
    _ = og.apply_diag_coulomb_evolution(vec, ham.J[0], DT, NORB, NELEC)
    t_p = time.perf_counter() - t0
    t_rot = d / R_c * t_c + 2 * d / R_g * t_g
    t_step = (2 * L + 1) * t_rot + L * t_p
    out = {
        "value": t_step,
        "unit": "s per DF Trotter step",
        "cores": int(max(workers, blas_threads)),
        "kind": "oracle",
        "sample": (f"{R_c} rows of the compound matrix C_8(U) ({R_c}x{d} 8x8 float64 determinants over {workers} "
                   f"processes, {t_c:.1f} s), {R_g}x{d} by {d}x{d} real products with Re and Im of the state "
                   f"({t_g:.1f} s on {blas_threads} BLAS threads), one full diagonal-Coulomb phase ({t_p:.1f} s); "
                   f"scaled to {2 * L + 1} rotations + {L} phases per step"),
    }
    golden = os.path.join(ROOT, "tests", "golden", "df_trotter_n16.txt")
    if os.path.exists(golden):
        with open(golden) as fh:
            for line in fh:
                if line.startswith("step_seconds"):
                    _, secs, ncores = line.split()
                    out["measured_whole_step"] = {"s": float(secs), "cores": int(ncores),
                                                  "where": "the build host (8 cores), once, for the stored "
                                                           "oracle result of this step"}
    if hubbard_small is not None:
        # the Trotter-error leg's small lattice, whole, in the oracle
        from oracle import hamiltonian as oh
        sx, sy = hubbard_small
        norb, nelec = sx * sy, synth.hubbard_filling(sx, sy)
        v = synth.random_state(synth.rng(0), ost.dim(norb, nelec[0]), ost.dim(norb, nelec[1]))
        t0 = time.perf_counter()
        err = oh.trotter_error(v, synth.hubbard_2d(sx, sy), 1.0, norb, nelec, 2, 1)
        out["trotter_error_hubbard_small"] = {"s": round(time.perf_counter() - t0, 3), "error": err,
                                              "workload": f"hubbard_2d {sx}x{sy} nelec={nelec} T=1.0: exact "
                                                          "evolution + S_1 with 2 steps + distance"}
    return out


def time_df_step(ffx, torch, ham, vec_np, dtype, steps, warmup, norb=NORB, nelec=NELEC, vec_dev=None):
    """Mean time per S_0 step over `steps` steps after `warmup` (HIP events on the working stream, one per
    step boundary, so the median and interquartile range of the single steps come out too), then the live
    per-launch timing of the kernel families over one more step."""
    dev = torch.device("cuda:0")
    vec = vec_dev if vec_dev is not None else torch.from_numpy(vec_np).to(dtype).to(dev)
    plan = ffx.get_plan(norb, nelec, dtype, 0)
    stream = torch.cuda.current_stream(dev)

    def step():
        ffx.simulate_trotter_double_factorized(vec, ham, DT, norb, nelec, n_steps=1, order=0, out=vec)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    t_wall = time.perf_counter()
    ev[0].record(stream)
    for k in range(steps):
        step()
        ev[k + 1].record(stream)
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_wall
    ms = ev[0].elapsed_time(ev[-1]) / steps
    per = np.array([ev[k].elapsed_time(ev[k + 1]) for k in range(steps)])
    stats = {"median_ms": float(np.median(per)), "iqr_ms": float(np.percentile(per, 75) - np.percentile(per, 25))}
    norm = float(torch.linalg.vector_norm(vec.to(torch.complex128) if vec.dtype != torch.complex128 else vec))

    # live per-launch timing of the kernel families over one more step
    plan.timing(True)
    step()
    torch.cuda.synchronize()
    fam = {}
    for kind, kname in ((2, "plane_pass"), (1, "seg_pass"), (0, "win_pass")):
        for spin, sname in ((0, "alpha"), (1, "beta")):
            kms, n, alg, slots = plan.timing_read(kind, spin)
            if n:
                fam[f"{kname}_{sname}"] = {"launches": n, "total_ms": kms, "avg_ms": kms / n,
                                           "alg_bytes": alg, "valu_slots": slots}
    plan.timing(False)
    del vec
    return ms, t_wall, norm, fam, plan.state_bytes, stats


def n18_timing(ffx, torch, synth, dtype, steps=3, warmup=1):
    """One S_0 step at norb = 18, (9, 9), L = 18 (48620 x 48620, 37.8 GB complex128), dt = 0.1, from a
    random normalized state drawn on the device (seeded torch generator); `steps` timed steps after `warmup`,
    and per kernel family two HBM rates against the 8 TB/s peak: `alg_GBps` counts 2 S per rotation side
    (one read and one write of the state per spin sweep of an orbital rotation, split over the passes by
    their share of the rotations), `moved_GBps` one read and one write of the whole state per launch (a
    segment pass visits every segment of every row; a window pass every class that holds some but not all
    of the window's orbitals, all but about 1 % of the state here)."""
    norb, nelec, nt = 18, (9, 9), 18
    ham = synth.df_hamiltonian(synth.rng(5), norb, nt)
    d = synth.dim(norb, 9)
    g = torch.Generator(device="cuda:0")
    g.manual_seed(5)
    vec = torch.randn((d, d), dtype=dtype, device="cuda:0", generator=g)
    vec /= torch.linalg.vector_norm(vec)
    ms, _, norm, fam, sb, stats = time_df_step(ffx, torch, ham, None, dtype, steps, warmup, norb, nelec,
                                               vec_dev=vec)
    del vec
    out = {"ms_per_step": ms, **stats, "state_bytes": sb, "final_norm": norm, "families": {}}
    for k, v in fam.items():
        gbs = v["alg_bytes"] / (v["total_ms"] * 1e-3) / 1e9
        moved = v["launches"] * 2 * sb / (v["total_ms"] * 1e-3) / 1e9
        out["families"][k] = {"launches": v["launches"], "avg_ms": round(v["avg_ms"], 3),
                              "alg_GBps": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
                              "moved_GBps": round(moved, 1), "moved_frac": round(moved / HBM_PEAK_GBS, 4)}
    ffx._plan_cached.cache_clear()
    torch.cuda.empty_cache()
    return out


KERNELS = {"plane_pass": "k_seg_pass_planes (rows as two planes; alpha and beta column spins)",
           "seg_pass": "k_seg_pass (alpha and beta column spins)"}


def roofline(fam, dtype_name, state_bytes, rotations_per_step):
    """Roofline of the dominant kernel of the step (the family of segment passes with the most kernel time:
    the plane passes for complex128 at 16 orbitals, the segment passes otherwise), and the HBM bytes of a whole
    step: the passes' algorithmic 2 S each and their counter-measured bytes, against the 4 S per orbital
    rotation of one read and one write of the state per spin sweep."""
    groups = {}
    for g in KERNELS:
        rows = [v for k, v in fam.items() if k.startswith(g)]
        if rows:
            groups[g] = {"n": sum(v["launches"] for v in rows), "ms": sum(v["total_ms"] for v in rows),
                         "slots": sum(v["valu_slots"] for v in rows)}
    dom = max(groups, key=lambda g: groups[g]["ms"])
    n, tot_ms, slots = groups[dom]["n"], groups[dom]["ms"], groups[dom]["slots"]
    sec = tot_ms / n * 1e-3
    # ALU: algorithmic VALU slots (8 per rotated amplitude pair for real rotations,
    # 12 for complex) as FMA-equivalent flops against the vector peak of the type
    alu_peak = 78.6 if dtype_name == "c128" else 157.3
    alu = 2.0 * slots / n / sec / 1e12
    # HBM: a segment pass reads and writes the whole state once
    hbm_bytes = 2.0 * state_bytes
    hbm = hbm_bytes / sec / 1e9
    if alu / alu_peak >= hbm / HBM_PEAK_GBS:
        r = {"bound": "alu", "achieved": round(alu, 3), "peak": alu_peak, "unit": "TFLOP/s",
             "frac": round(alu / alu_peak, 4)}
    else:
        r = {"bound": "hbm", "achieved": round(hbm, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
             "frac": round(hbm / HBM_PEAK_GBS, 4)}
    key = {"plane_pass": f"{dtype_name}_planes", "seg_pass": dtype_name}
    tr = committed_traffic(key[dom])
    measured = [committed_traffic(key[g]) for g in groups]
    step_launch_bytes = sum(groups[g]["n"] for g in groups) * hbm_bytes
    r.update({
        "traffic": tr,
        # measured HBM bytes per launch (when the committed counters match these kernels, else the
        # algorithmic 2 S) over the average launch time, against the 8 TB/s peak
        "hbm_frac": round((tr if tr else hbm_bytes) / sec / 1e9 / HBM_PEAK_GBS, 4),
        "kernel": KERNELS[dom],
        "per_step": {
            "launches": {g: groups[g]["n"] for g in groups},
            "kernel_ms": {g: round(groups[g]["ms"], 3) for g in groups},
            "alg_bytes_2S_per_launch": step_launch_bytes,
            "reference_bytes_4S_per_rotation": 4.0 * state_bytes * rotations_per_step,
            "measured_bytes": (sum(groups[g]["n"] * m for g, m in zip(groups, measured))
                               if all(m is not None for m in measured) else None),
        },
        "avg_launch_ms": round(tot_ms / n, 4),
        "launches_per_step": n,
        "valu_slots_per_launch": slots / n,
        "alg_hbm_bytes_per_launch": hbm_bytes,
        "hbm_GBps": round(hbm, 1),
        "alu_TFLOPs": round(alu, 3),
        "kernel_sources_sha256": kernel_source_hash(),
        "families": fam,
    })
    return r


def lucj_timing(ffx, torch, synth, dtype, with_fd):
    wl = synth.workload_lucj(NORB, LUCJ_REPS, L, seed=0)
    p, ham = wl.data["params"], wl.data["ham"]
    ffx.lucj_energy_grad(p, ham, NORB, NELEC, LUCJ_REPS, dtype=dtype)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e, g = ffx.lucj_energy_grad(p, ham, NORB, NELEC, LUCJ_REPS, dtype=dtype)
    t_adj = time.perf_counter() - t0
    out = {"energy": e, "adjoint_s": t_adj, "n_params": int(g.size)}
    if not with_fd:
        return out
    plan = ffx.get_plan(NORB, NELEC, dtype, 0)
    psi = torch.empty((plan.dim_a, plan.dim_b), dtype=dtype, device="cuda:0")

    def energy(q):
        ffx.apply_lucj(q, NORB, NELEC, LUCJ_REPS, dtype=dtype, out=psi, plan=plan)
        return ffx.df_energy(psi, ham, NORB, NELEC, plan=plan)

    idx = synth.fd_indices(g.size, 20)
    energy(p)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fd = []
    for i in idx:
        qp, qm = p.copy(), p.copy()
        qp[i] += FD_H
        qm[i] -= FD_H
        fd.append((energy(qp) - energy(qm)) / (2 * FD_H))
    t_fd = time.perf_counter() - t0
    out.update({"fd_params": len(idx), "fd_s": t_fd, "fd_all_params_s_extrapolated": t_fd / len(idx) * g.size,
                "fd_h": FD_H, "max_abs_adjoint_minus_fd": float(np.max(np.abs(np.array(fd) - g[idx]))),
                "adjoint_speedup_vs_fd_all": t_fd / len(idx) * g.size / t_adj})
    return out


def chain_timing(ffx, torch, synth, ham, vec_np, dtype):
    """Energy after one S_0 step of the metric's DF Hamiltonian (norb = 16, L = 16, dt = 0.1) under a second
    DF Hamiltonian as the observable (seed 1), and its adjoint gradient with respect to h, every J_t and every
    U_t generator: one call, after one warm-up call."""
    obs = synth.df_hamiltonian(synth.rng(1), NORB, L)
    vec = torch.from_numpy(vec_np).to(dtype).to("cuda:0")
    ffx.df_chain_energy_grad(vec, ham, obs, DT, 1, NORB, NELEC)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e, g = ffx.df_chain_energy_grad(vec, ham, obs, DT, 1, NORB, NELEC)
    t = time.perf_counter() - t0
    n_params = int(g["h"].size + g["J"].size + g["U"].size)
    del vec
    return {"energy": e, "s": round(t, 4), "n_params": n_params}


def batched_timing(ffx, torch, synth, dtype):
    """Config-4 workload: 256 sectors (norb in {8, 10, 12}, n in {norb/2 - 1, norb/2}), each with its
    own LUCJ (n_reps = 2) and DF Hamiltonian (L = norb): energies and adjoint gradients of all of them."""
    w = synth.workload_batched(256, seed=0, n_reps=2)
    b = ffx.Batch([(x.norb, x.nelec) for x in w], dtype=dtype)
    args = ([x.data["params"] for x in w], [x.data["ham"] for x in w], 2)
    tuned = b.tune(*args)  # task size and stage depth for this batch (a few seconds)
    b.lucj_energy_grad(*args)
    torch.cuda.synchronize()
    runs = []
    for _ in range(3):
        b.lucj_energy_grad(*args)
        runs.append(b.timing())
    best = min(runs, key=lambda r: r["device_ms"])
    # the same batch as one cooperative launch, for comparison
    b.single_launch(True)
    b.lucj_energy_grad(*args)
    torch.cuda.synchronize()
    runs1 = []
    for _ in range(3):
        b.lucj_energy_grad(*args)
        runs1.append(b.timing())
    b.single_launch(False)
    best1 = min(runs1, key=lambda r: r["device_ms"])
    return {"device_ms": best["device_ms"], "call_ms": best["call_ms"], "launches": best["launches"],
            "tuned": {"target_elems": tuned[0], "stage_rots": tuned[1]},
            "single_cooperative_launch": {"device_ms": best1["device_ms"], "call_ms": best1["call_ms"],
                                          "launches": best1["launches"]},
            "config": b.info(), "amplitudes": int(sum(synth.dim(x.norb, x.nelec[0]) * synth.dim(x.norb, x.nelec[1])
                                                      for x in w))}


def hubbard_timing(ffx, torch, synth, nx, ny, time_T=1.0, oracle_side=(4, 4)):
    """Trotter-error workload (Sec. 6.2): 2D Hubbard model t = 1, U = 8 on an nx x ny lattice periodic in x,
    1/8 filling, from a random unit state (seed 0), complex128: one Hamiltonian action, the exact evolution
    exp(-i H T) (Chebyshev expansion, tol 1e-12), Trotter runs of orders 1 and 2 against it, and the live
    per-launch timing of the kernel families over one S_1 step.  Beside it, the same measurement
    at the small lattice `oracle_side` on the GPU and in the oracle."""
    from math import comb
    dev = torch.device("cuda:0")
    dtype = torch.complex128
    norb, nelec = nx * ny, synth.hubbard_filling(nx, ny)
    ham = synth.hubbard_2d(nx, ny)
    plan = ffx.get_plan(norb, nelec, dtype, 0)
    da, db = comb(norb, nelec[0]), comb(norb, nelec[1])
    g = torch.Generator(device=dev)
    g.manual_seed(0)
    vec = torch.randn((da, db), dtype=dtype, device=dev, generator=g)
    vec /= torch.linalg.vector_norm(vec)
    out = torch.empty_like(vec)
    ffx.apply_df_hamiltonian(vec, ham, norb, nelec, out=out, plan=plan)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ffx.apply_df_hamiltonian(vec, ham, norb, nelec, out=out, plan=plan)
    torch.cuda.synchronize()
    t_h = time.perf_counter() - t0
    plan.timing(True)
    out.copy_(vec)
    ffx.simulate_trotter_double_factorized(vec, ham, time_T, norb, nelec, n_steps=1, order=1, out=out, plan=plan)
    torch.cuda.synchronize()
    fam = {}
    for kind, kname in ((1, "seg_pass"), (0, "win_pass")):
        for spin, sname in ((0, "alpha"), (1, "beta")):
            kms, n, alg, slots = plan.timing_read(kind, spin)
            if n:
                fam[f"{kname}_{sname}"] = {"launches": n, "total_ms": round(kms, 3), "avg_ms": round(kms / n, 4),
                                           "alu_TFLOPs": round(2.0 * slots / (kms * 1e-3) / 1e12, 3),
                                           "alg_GBps": round(alg / (kms * 1e-3) / 1e9, 1)}
    plan.timing(False)
    del out
    exact = vec.clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, k = ffx.evolve_exact(vec, ham, time_T, norb, nelec, out=exact, plan=plan)
    torch.cuda.synchronize()
    t_exact = time.perf_counter() - t0
    runs = []
    approx = torch.empty_like(vec)
    h_dc, Jaa, Jab, Jbb = synth.hubbard_2d_diag_coulomb(nx, ny)
    for order, n in ((1, 2), (2, 1)):
        for route in ("diag_coulomb", "df"):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if route == "df":
                ffx.simulate_trotter_double_factorized(vec, ham, time_T, norb, nelec, n_steps=n, order=order,
                                                       out=approx, plan=plan)
            else:
                ffx.simulate_trotter_diag_coulomb(vec, h_dc, Jaa, time_T, norb, nelec, J_ab=Jab, J_bb=Jbb, n_steps=n,
                                                  order=order, out=approx, plan=plan)
            torch.cuda.synchronize()
            t_tr = time.perf_counter() - t0
            runs.append({"route": route, "order": order, "n_steps": n, "s": round(t_tr, 4),
                         "s_per_step": round(t_tr / n, 4),
                         "error": ffx.state_distance(approx, exact, norb, nelec, plan=plan)})
    res = {"workload": f"hubbard_2d {nx}x{ny} periodic_x t=1 U=8 nelec={nelec} T={time_T} state=c128 {da}x{db}",
           "state_bytes": plan.state_bytes, "h_action_s": round(t_h, 4),
           "exact": {"s": round(t_exact, 3), "n_matvec": k, "tol": 1e-12}, "trotter": runs, "families": fam}
    del vec, exact, approx
    ffx._plan_cached.cache_clear()
    del plan
    torch.cuda.empty_cache()
    # the same measurement at a size the oracle finishes (the oracle side runs in the cpu_baseline leg)
    sx, sy = oracle_side
    norb, nelec = sx * sy, synth.hubbard_filling(sx, sy)
    ham = synth.hubbard_2d(sx, sy)
    v = synth.random_state(synth.rng(0), comb(norb, nelec[0]), comb(norb, nelec[1]))
    vd = torch.from_numpy(v).to(dev)
    ffx.evolve_exact(vd, ham, time_T, norb, nelec)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ex, _ = ffx.evolve_exact(vd, ham, time_T, norb, nelec)
    ap_ = ffx.simulate_trotter_double_factorized(vd, ham, time_T, norb, nelec, n_steps=2, order=1)
    err_gpu = ffx.state_distance(ap_, ex, norb, nelec)
    t_gpu = time.perf_counter() - t0
    res["small"] = {"workload": f"hubbard_2d {sx}x{sy} nelec={nelec} T={time_T}, state synth.random_state seed 0: "
                                "exact evolution + S_1 with 2 steps + distance",
                    "s": round(t_gpu, 4), "error": err_gpu}
    return res


def dense_vs_givens(ffx, torch, synth, reps=20):
    """One orbital rotation (complex Haar U, both spins) at half filling, complex128, state resident: the
    Givens sweeps (ffx_apply_orbital_rotation) against the dense compound-matrix form on the FP64 matrix
    cores (ffx_apply_orbital_rotation_dense: compound matrices built on the device, two complex products).
    Mean of `reps` calls after two warm-ups, HIP events on the launch stream; algorithmic flops
    20 n (N - n) d^2 (Givens, both spins, complex s) and 16 d^3 (dense, two complex GEMMs)."""
    from math import comb
    dev = torch.device("cuda:0")
    out = {}
    for norb in (8, 10, 12, 14):
        n = norb // 2
        d = comb(norb, n)
        r = synth.rng([73, norb])
        vec = torch.from_numpy(synth.random_state(r, d, d)).to(dev)
        U = synth.random_unitary(r, norb)
        res = {"d": d}
        # the Givens sweeps on a plan that never takes the dense form (small sectors otherwise would)
        os.environ["FFX_DENSE"] = "0"
        try:
            gplan = ffx.Plan(norb, (n, n), torch.complex128)
        finally:
            del os.environ["FFX_DENSE"]
        dplan = ffx.get_plan(norb, (n, n), torch.complex128, 0)
        for name, fn, plan in (("givens", ffx.apply_orbital_rotation, gplan),
                               ("dense_mfma", ffx.apply_orbital_rotation_dense, dplan)):
            for _ in range(2):
                fn(vec, U, norb, (n, n), out=vec, plan=plan)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                fn(vec, U, norb, (n, n), out=vec, plan=plan)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            flop = 20.0 * n * (norb - n) * d * d if name == "givens" else 16.0 * d ** 3
            res[name] = {"ms": round(ms, 5), "alg_TFLOPs": round(flop / (ms * 1e-3) / 1e12, 3)}
        res["dense_over_givens"] = round(res["dense_mfma"]["ms"] / res["givens"]["ms"], 3)
        out[f"norb{norb}_({n},{n})"] = res
        del vec
    torch.cuda.empty_cache()
    return out


def table1_timing(ffx, torch, synth):
    """Time per call of the Table 1 gates, the Slater-determinant state and a UCJ forward pass (n_reps = 3,
    per-spin rotations, full J) at norb = 16, (8, 8), complex128, state resident on the device."""
    dev = torch.device("cuda:0")
    r = synth.rng(7)
    vec = torch.from_numpy(synth.random_state(r, 12870, 12870)).to(dev)
    plan = ffx.get_plan(NORB, NELEC, torch.complex128, 0)
    M = synth.random_hermitian(r, NORB, 0.5)
    R = 3
    U = np.array([synth.random_unitary(r, NORB) for _ in range(R)])
    Ub = np.array([synth.random_unitary(r, NORB) for _ in range(R)])
    J = np.array([synth.random_symmetric(r, NORB, 0.3) for _ in range(R)])
    calls = {
        "num_interaction": lambda: ffx.apply_num_interaction(vec, 0.3, 5, 0, NORB, NELEC, out=vec, plan=plan),
        "num_num_interaction": lambda: ffx.apply_num_num_interaction(vec, 0.3, 5, 0, 9, 1, NORB, NELEC, out=vec,
                                                                     plan=plan),
        "givens_rotation_adjacent": lambda: ffx.apply_givens_rotation(vec, 0.3, 7, 8, 1, NORB, NELEC, out=vec,
                                                                      plan=plan),
        "givens_rotation_0_15": lambda: ffx.apply_givens_rotation(vec, 0.3, 0, 15, 0, NORB, NELEC, out=vec, plan=plan),
        "tunneling_interaction": lambda: ffx.apply_tunneling_interaction(vec, 0.3, 3, 4, 0, NORB, NELEC, out=vec,
                                                                         plan=plan),
        "quad_ham_evolution": lambda: ffx.apply_quad_ham_evolution(vec, M, 0.1, NORB, NELEC, out=vec, plan=plan),
        "slater_determinant": lambda: ffx.slater_determinant(NORB, NELEC, U=U[0], U_b=Ub[0], out=vec, plan=plan),
        "ucj_n_reps_3": lambda: ffx.apply_ucj(NORB, NELEC, U, J, U_b=Ub, J_ab=J, J_bb=J, out=vec, plan=plan),
    }
    ua = r.random(100000)
    us = (r.random((100000, 8)), r.random((100000, 8)))
    calls["sample_state_1e5"] = lambda: ffx.sample_state(vec, ua, NORB, NELEC, plan=plan)
    calls["sample_slater_1e5"] = lambda: ffx.sample_slater(NORB, NELEC, us[0], us[1], U=U[0], U_b=Ub[0], plan=plan)
    out = {}
    for name, f in calls.items():
        f()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            f()
        torch.cuda.synchronize()
        out[name + "_ms"] = round((time.perf_counter() - t0) / 3 * 1e3, 3)
    del vec
    return out


def _event_times(torch, call, reps, warmup):
    """Milliseconds per call of `call` (HIP events on the current stream between consecutive calls):
    median, interquartile range and mean over `reps` calls after `warmup`."""
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        call()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
    ev[0].record(stream)
    for k in range(reps):
        call()
        ev[k + 1].record(stream)
    torch.cuda.synchronize()
    per = np.array([ev[k].elapsed_time(ev[k + 1]) for k in range(reps)])
    return {"median_ms": round(float(np.median(per)), 5),
            "iqr_ms": round(float(np.percentile(per, 75) - np.percentile(per, 25)), 5),
            "mean_ms": round(float(per.mean()), 5)}


def config2_timing(ffx, torch, synth, reps=20, warmup=3):
    """DF Trotter at norb = 14, (7, 7), L = 14 (h ~ N(0, 0.5), U_t real orthogonal, J_t ~ N(0, 0.1)), dt = 0.1:
    two S_0 steps from the Hartree-Fock state per call (out of place, so every call starts from it), in both
    precisions.  The 3432 x 3432 state (188 / 94 MB) stays in the 256 MB Infinity Cache, so the figure is
    time, not an HBM rate."""
    dev = torch.device("cuda:0")
    w = synth.workload_df_trotter(14, 14, seed=0, start="hf", dt=0.1, n_steps=2)
    ham = w.data["ham"]
    out = {"workload": "df_trotter norb=14 nelec=(7,7) L=14 dt=0.1 order=0, 2 steps per call from Hartree-Fock"}
    for name, dtype in (("c128", torch.complex128), ("c64", torch.complex64)):
        v0 = torch.from_numpy(w.data["vec"]).to(dtype).to(dev)
        vec = torch.empty_like(v0)
        plan = ffx.get_plan(14, (7, 7), dtype, 0)

        def call():
            ffx.simulate_trotter_double_factorized(v0, ham, 0.2, 14, (7, 7), n_steps=2, order=0, out=vec,
                                                   plan=plan)

        t = _event_times(torch, call, reps, warmup)
        out[name] = {"s_per_step_median": round(t["median_ms"] / 2e3, 7), "ms_per_call": t,
                     "final_norm": float(torch.linalg.vector_norm(vec.to(torch.complex128)))}
        del v0, vec
    return out


def fig2_shapes(ffx, torch, synth, reps=20, warmup=3, norbs=range(4, 17, 2)):
    """Time per call, in the shape of the paper's Fig. 2 benchmarks (Sec. 5.2), complex128 state resident on
    the device: quadratic-Hamiltonian evolution (random Hermitian M, t = 1), diagonal-Coulomb evolution
    (random symmetric J, t = 1) and three S_0 steps of a DF Trotter simulation of a Hamiltonian with three
    two-body terms (dt = 0.1), for norb = 4, 6, ..., 16 at half filling (norb / 2 electrons per spin) and at
    quarter filling (norb // 4 per spin).  Median and interquartile range of `reps` calls."""
    dev = torch.device("cuda:0")
    out = {"workload": "Fig. 2 shapes: quad_ham_evolution, diag_coulomb_evolution, df_trotter 3 steps L=3; "
                       "c128; norb 4..16; half and quarter filling"}
    for filling, nfun in (("half", lambda n: n // 2), ("quarter", lambda n: n // 4)):
        rows = {}
        for norb in norbs:
            n = nfun(norb)
            nelec = (n, n)
            r = synth.rng(100 + norb)
            d = synth.dim(norb, n)
            vec = torch.from_numpy(synth.random_state(r, d, d)).to(dev)
            plan = ffx.get_plan(norb, nelec, torch.complex128, 0)
            M = synth.random_hermitian(r, norb, 0.5)
            J = synth.random_symmetric(r, norb, 0.3)
            ham = synth.df_hamiltonian(r, norb, 3)
            calls = {
                "quad_ham_evolution": lambda: ffx.apply_quad_ham_evolution(vec, M, 1.0, norb, nelec, out=vec,
                                                                           plan=plan),
                "diag_coulomb_evolution": lambda: ffx.apply_diag_coulomb_evolution(vec, J, 1.0, norb, nelec,
                                                                                   out=vec, plan=plan),
                "df_trotter_3_steps_L3": lambda: ffx.simulate_trotter_double_factorized(
                    vec, ham, 0.3, norb, nelec, n_steps=3, order=0, out=vec, plan=plan),
            }
            rows[f"norb{norb}_({n},{n})"] = {k: _event_times(torch, f, reps, warmup) for k, f in calls.items()}
            del vec
        out[filling] = rows
    torch.cuda.empty_cache()
    return out


def copy_calibration(torch):
    """Plain device copies of a known size for scaling the HBM byte counters."""
    n = 1 << 27  # 2^27 complex64 = 1 GiB
    a = torch.zeros(n, dtype=torch.complex64, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_read": n * 8, "copy_calibration_bytes_written": n * 8,
                      "copies": 3}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--dtype", choices=["c128", "c64"], default="c128")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-lucj", action="store_true")
    ap.add_argument("--no-other-dtype", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-hubbard", action="store_true")
    ap.add_argument("--no-table1", action="store_true")
    ap.add_argument("--no-n18", action="store_true")
    ap.add_argument("--hubbard-y", type=int, default=8, help="lattice 4 x y of the Trotter-error leg")
    ap.add_argument("--hubbard-only", action="store_true", help="run only the Trotter-error leg (for profiling)")
    ap.add_argument("--table1-only", action="store_true",
                    help="run only the Table 1 gates and sampling leg (for profiling)")
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--no-dense", action="store_true")
    ap.add_argument("--dense-only", action="store_true",
                    help="run only the dense-vs-Givens rotation leg (for profiling)")
    ap.add_argument("--n18-only", action="store_true",
                    help="run only the 18-orbital DF step in the --dtype precision (for profiling)")
    ap.add_argument("--no-config2", action="store_true")
    ap.add_argument("--no-fig2", action="store_true")
    ap.add_argument("--context-only", action="store_true",
                    help="run only the norb=14 DF leg and the Fig. 2-shaped legs")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the state of this workload fits one MI355X and the build has no "
              "multi-GPU path; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2605_03123_amd import ffx, synth

    if args.copy_calibration:
        copy_calibration(torch)
        return

    if args.hubbard_only:
        print(json.dumps({"trotter_error_hubbard": hubbard_timing(ffx, torch, synth, 4, args.hubbard_y)}), flush=True)
        return
    if args.table1_only:
        print(json.dumps({"table1_gates_n16_c128": table1_timing(ffx, torch, synth)}), flush=True)
        return
    if args.dense_only:
        print(json.dumps({"rotation_dense_vs_givens_c128": dense_vs_givens(ffx, torch, synth)}), flush=True)
        return
    if args.n18_only:
        dt = torch.complex128 if args.dtype == "c128" else torch.complex64
        print(json.dumps({"df_step_n18": {args.dtype: n18_timing(ffx, torch, synth, dt, args.steps, args.warmup)}}),
              flush=True)
        return
    if args.context_only:
        print(json.dumps({"df_trotter_n14": config2_timing(ffx, torch, synth),
                          "fig2_shapes": fig2_shapes(ffx, torch, synth)}), flush=True)
        return

    types = {"c128": torch.complex128, "c64": torch.complex64}
    w = synth.workload_df_trotter(NORB, L, seed=0, start="random", dt=DT)
    ham, vec_np = w.data["ham"], w.data["vec"]
    ms, t_wall, norm, fam, state_bytes, stats = time_df_step(ffx, torch, ham, vec_np, types[args.dtype],
                                                              args.steps, args.warmup)
    out = {
        "metric": "s per DF Trotter step (norb=16, nelec=(8,8), L=16, S_0, dt=0.1)",
        "value": ms / 1e3,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "ms_per_step_median": stats["median_ms"],
        "ms_per_step_iqr": stats["iqr_ms"],
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.dtype == "c128" else "f32",
        "data": "synthetic (seeded random DF Hamiltonian and random normalized state)",
        "config": {"workload": f"df_trotter_step norb=16 nelec=(8,8) L=16 dt=0.1 order=0 "
                               f"state={args.dtype} 12870x12870", "state_bytes": state_bytes,
                   "wall_s_timed": round(t_wall, 3), "final_norm": norm},
        "roofline": roofline(fam, args.dtype, state_bytes, L + 1),
    }
    if not args.no_other_dtype:
        other = "c64" if args.dtype == "c128" else "c128"
        ms2, _, norm2, fam2, sb2, st2 = time_df_step(ffx, torch, ham, vec_np, types[other], args.steps,
                                                     args.warmup)
        rf2 = roofline(fam2, other, sb2, L + 1)
        rf2.pop("families")
        out[f"df_step_{other}"] = {"ms_per_step": ms2, "ms_per_step_median": st2["median_ms"],
                                   "ms_per_step_iqr": st2["iqr_ms"], "final_norm": norm2, "roofline": rf2}
    if not args.no_lucj:
        out["lucj_energy_grad"] = {
            "workload": f"lucj norb=16 nelec=(8,8) n_reps={LUCJ_REPS} L={L} params~N(0,0.1)",
            "c128": lucj_timing(ffx, torch, synth, torch.complex128, True),
            "c64": lucj_timing(ffx, torch, synth, torch.complex64, False),
        }
    if not args.no_lucj:
        out["df_chain_energy_grad"] = {
            "workload": "E = Re<psi_1|H_obs|psi_1>, psi_1 = S_0(0.1) psi_0 (metric's DF Hamiltonian and state), "
                        "H_obs = DF L=16 seed 1; adjoint gradient in h, J_t, U_t",
            "c128": chain_timing(ffx, torch, synth, ham, vec_np, torch.complex128),
            "c64": chain_timing(ffx, torch, synth, ham, vec_np, torch.complex64),
        }
    if not args.no_batched:
        out["batched_lucj_energy_grad"] = {
            "workload": "256 sectors, norb in {8,10,12}, n in {norb/2-1, norb/2}, LUCJ n_reps=2, DF L=norb "
                        "(energies + adjoint gradients; one launch per pass kind of each level after tuning, the single cooperative launch beside it)",
            "c64": batched_timing(ffx, torch, synth, torch.complex64),
            "c128": batched_timing(ffx, torch, synth, torch.complex128),
        }
    if not args.no_n18:
        out["df_step_n18"] = {"workload": "df_trotter_step norb=18 nelec=(9,9) L=18 dt=0.1 order=0, random state",
                              "c128": n18_timing(ffx, torch, synth, torch.complex128),
                              "c64": n18_timing(ffx, torch, synth, torch.complex64)}
    if not args.no_config2:
        out["df_trotter_n14"] = config2_timing(ffx, torch, synth)
    if not args.no_fig2:
        out["fig2_shapes"] = fig2_shapes(ffx, torch, synth)
    if not args.no_table1:
        out["table1_gates_n16_c128"] = table1_timing(ffx, torch, synth)
    if not args.no_dense:
        out["rotation_dense_vs_givens_c128"] = dense_vs_givens(ffx, torch, synth)
    if not args.no_hubbard:
        out["trotter_error_hubbard"] = hubbard_timing(ffx, torch, synth, 4, args.hubbard_y)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(ham, vec_np, synth, None if args.no_hubbard else (4, 4))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
