"""Benchmark: seconds per double-factorized Trotter step at norb = 16, (8, 8).

    python bench.py [--steps K] [--warmup W] [--dtype c128|c64] [--no-cpu-baseline] [--lucj]

Workload: one first-order (S_0) Trotter step, dt = 0.1, of a DF Hamiltonian
with L = 16 terms (h ~ sym N(0, 0.5); U_t real orthogonal from QR; J_t ~ sym
N(0, 0.1)) on a random normalized 12870 x 12870 state, seed 0.  The state is
resident in HBM before timing; W untimed steps, then K timed steps bracketed by
device synchronization, timed with HIP events on the working stream.

Prints ONE JSON line with the metric, a roofline object for the dominant
kernel family (the Givens window passes; per-launch durations measured live
with HIP events on the launch stream) and the oracle timed on a bounded sample
of the same step.
"""
from __future__ import annotations

import argparse
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


def cpu_baseline(ham, vec: np.ndarray) -> dict:
    """Time the oracle on a bounded sample of one Trotter step and scale to a whole step.

    The oracle applies each orbital rotation as Gamma' = C(U) Gamma C(U)^T with
    the compound matrix C(U) built from all dim^2 minors, and each diagonal
    Coulomb phase over the whole state.  Sample: R_c rows of C(U) (R_c * dim
    determinants), the product of R_g rows of C(U) with Gamma, and one full
    diagonal Coulomb phase.  Scaled: per rotation dim/R_c * t_C + 2 dim/R_g * t_G;
    per step (2L + 1) rotations and L phases (the oracle does not merge rotations).
    """
    from oracle import gates as og
    from oracle import sampled
    from oracle import strings as ost
    try:
        from threadpoolctl import threadpool_info
        blas_threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        blas_threads = len(os.sched_getaffinity(0))
    d = ost.dim(NORB, NELEC[0])
    U = np.asarray(ham.U[0]).conj().T
    ost.occupied_lists(NORB, NELEC[0])
    R_c, R_g = 128, 512
    t0 = time.perf_counter()
    rows = np.array([sampled.compound_row(U, NELEC[0], i) for i in range(R_c)])
    t_c = time.perf_counter() - t0
    A = np.vstack([rows] * (R_g // R_c))
    t0 = time.perf_counter()
    _ = A @ vec
    t_g = time.perf_counter() - t0
    t0 = time.perf_counter()
    _ = og.apply_diag_coulomb_evolution(vec, ham.J[0], DT, NORB, NELEC)
    t_p = time.perf_counter() - t0
    t_rot = d / R_c * t_c + 2 * d / R_g * t_g
    t_step = (2 * L + 1) * t_rot + L * t_p
    return {
        "value": t_step,
        "unit": "s per DF Trotter step",
        "cores": int(blas_threads),
        "kind": "oracle",
        "sample": (f"{R_c} rows of the compound matrix C_8(U) ({R_c}x{d} 8x8 determinants, {t_c:.1f} s), "
                   f"{R_g}x{d} by {d}x{d} complex product ({t_g:.1f} s), one full diagonal-Coulomb phase "
                   f"({t_p:.1f} s); scaled to {2 * L + 1} rotations + {L} phases per step"),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--dtype", choices=["c128", "c64"], default="c128")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--lucj", action="store_true", help="also time LUCJ energy + adjoint gradient (n_reps=3)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the state of this workload fits one MI355X and the build has no "
              "multi-GPU path; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2605_03123_amd import ffx, synth

    dtype = torch.complex128 if args.dtype == "c128" else torch.complex64
    w = synth.workload_df_trotter(NORB, L, seed=0, start="random", dt=DT)
    ham, vec_np = w.data["ham"], w.data["vec"]
    dev = torch.device("cuda:0")
    vec = torch.from_numpy(vec_np).to(dtype).to(dev)
    plan = ffx.get_plan(NORB, NELEC, dtype, 0)
    stream = torch.cuda.current_stream(dev)

    def step():
        ffx.simulate_trotter_double_factorized(vec, ham, DT, NORB, NELEC, n_steps=1, order=0, out=vec)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t_wall = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_wall
    ms = e0.elapsed_time(e1) / args.steps
    norm = float(torch.linalg.vector_norm(vec.to(torch.complex128)))

    # live per-launch timing of the dominant kernels over one more step
    plan.timing(True)
    step()
    torch.cuda.synchronize()
    fam = {}
    for kind, kname in ((1, "seg_pass"), (0, "win_pass")):
        for spin, sname in ((0, "alpha"), (1, "beta")):
            kms, n, alg, slots = plan.timing_read(kind, spin)
            if n:
                fam[f"{kname}_{sname}"] = {"launches": n, "total_ms": kms, "avg_ms": kms / n,
                                           "alg_bytes": alg, "valu_slots": slots}
    plan.timing(False)
    dom = max(fam, key=lambda k: fam[k]["total_ms"])
    f = fam[dom]
    sec = f["avg_ms"] * 1e-3
    # ALU roofline: algorithmic VALU slots (8 per rotated pair for real rotations, 12 for complex)
    # as FMA-equivalent flops against the vector peak of the arithmetic type
    alu_peak = 78.6 if dtype == torch.complex128 else 157.3
    alu = 2.0 * f["valu_slots"] / f["launches"] / sec / 1e12
    # HBM roofline: a segment pass reads and writes the whole state once
    hbm_bytes = 2.0 * plan.state_bytes if dom.startswith("seg") else f["alg_bytes"] / f["launches"]
    hbm = hbm_bytes / sec / 1e9
    if alu / alu_peak >= hbm / HBM_PEAK_GBS:
        roofline = {"bound": "alu", "achieved": round(alu, 3), "peak": alu_peak, "unit": "TFLOP/s",
                    "frac": round(alu / alu_peak, 4)}
    else:
        roofline = {"bound": "hbm", "achieved": round(hbm, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(hbm / HBM_PEAK_GBS, 4)}
    roofline.update({
        "traffic": None,
        "kernel": f"k_{dom.rsplit('_', 1)[0]} ({dom.rsplit('_', 1)[1]} rotations)",
        "avg_launch_ms": round(f["avg_ms"], 4),
        "launches_per_step": f["launches"],
        "valu_slots_per_launch": f["valu_slots"] / f["launches"],
        "hbm_bytes_per_launch": hbm_bytes,
        "hbm_GBps": round(hbm, 1),
        "alu_TFLOPs": round(alu, 3),
        "families": fam,
    })

    out = {
        "metric": "s per DF Trotter step (norb=16, nelec=(8,8), L=16, S_0, dt=0.1)",
        "value": ms / 1e3,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if dtype == torch.complex128 else "f32",
        "data": "synthetic (seeded random DF Hamiltonian and random normalized state)",
        "config": {"workload": f"df_trotter_step norb=16 nelec=(8,8) L=16 dt=0.1 order=0 "
                               f"state={args.dtype} 12870x12870", "state_bytes": plan.state_bytes,
                   "wall_s_timed": round(t_wall, 3), "final_norm": norm},
        "roofline": roofline,
    }
    if args.lucj:
        wl = synth.workload_lucj(NORB, 3, L, seed=0)
        p = wl.data["params"]
        ffx.lucj_energy_grad(p, wl.data["ham"], NORB, NELEC, 3, dtype=dtype)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e, g = ffx.lucj_energy_grad(p, wl.data["ham"], NORB, NELEC, 3, dtype=dtype)
        out["lucj_energy_grad_s"] = time.perf_counter() - t0
        out["lucj_energy"] = e
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(ham, vec_np)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
