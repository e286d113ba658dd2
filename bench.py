"""Benchmark of the LES time step on one MI355X.

One step = one full time step of the moist anelastic LES (thermodynamics,
SGS viscosity, scalar and momentum predictors, radiation, Poisson RHS,
Chebyshev-weighted Jacobi solve to relative residual 1e-6, projection; two
predictor-corrector sub-iterations) on the synthetic stratocumulus workload
of 256 x 256 x 128 cells (35 m x 35 m x 5 m, dt 0.3 s, FP32 storage with
FP64 reductions and saturation adjustment).  Inputs are resident in HBM
before the timed region starts.

Prints one JSON line: Mcell-steps/s over the timed steps, Poisson seconds
per step, the roofline of the dominant kernel (the Chebyshev sweep) and the
FP64 CPU oracle timed on the host on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="C2")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-crop", type=int, default=128,
                    help="horizontal size of the crop the oracle's non-Poisson work is timed on")
    return ap.parse_args()


def sweep_bytes_per_cell(p):
    es = 8 if p["precision"] == "fp64" else 4
    # Chebyshev: read phi_m, phi_{m-1}, rhs; write phi_{m+1}.  Jacobi: 3 arrays.
    return (4 if p["poisson_scheme"] == "chebyshev" else 3) * es


def cpu_baseline(p, sweeps_per_step, crop):
    """Oracle (serial FP64 C, one thread) on a bounded sample: one step of
    the non-Poisson work on a crop x crop x nz sub-grid (one sweep per solve),
    scaled per cell to the full grid, plus 10 sweeps timed at the full grid,
    scaled by the GPU's measured sweeps per step."""
    import les_inputs as li
    import oracle

    nfull = p["nx"] * p["ny"] * p["nz"]
    pc = dict(p)
    pc["nx"] = pc["ny"] = min(crop, p["nx"])
    K = p["n_subiter"]
    st = li.initial_state(pc)
    t0 = time.perf_counter()
    oracle.step(pc, st, nsteps=1, replay=[1] * K)
    t_np = time.perf_counter() - t0
    ncrop = pc["nx"] * pc["ny"] * pc["nz"]
    rhs = li.random_field((p["nz"], p["ny"], p["nx"]), seed=3)
    nsw = 10
    t0 = time.perf_counter()
    oracle.poisson(p, rhs, fixed_sweeps=nsw)
    t_sw = (time.perf_counter() - t0) / nsw
    t_step = t_np * nfull / ncrop + sweeps_per_step * t_sw
    return {
        "value": nfull / t_step / 1e6,
        "unit": "Mcell-steps/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"one oracle step with one sweep per solve on a {pc['nx']}x{pc['ny']}x{pc['nz']} "
                   f"crop ({t_np:.1f} s, scaled per cell to {p['nx']}x{p['ny']}x{p['nz']}) plus "
                   f"{nsw} sweeps at full size ({t_sw * 1e3:.1f} ms/sweep) times the measured "
                   f"{sweeps_per_step:.0f} sweeps/step; extrapolated s/step {t_step:.1f}"),
    }


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the LES step is built and measured on a "
              "single MI355X (no multi-GPU decomposition in this build); use --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import les_inputs as li
    from paper_2301_04698_amd import les

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    p = li.workload(args.workload)
    ncell = p["nx"] * p["ny"] * p["nz"]
    sim = les.LES(p, li.initial_state(p), device="cuda:0")

    if args.warmup > 0:
        sim.step(args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc, st, recs = sim.step(args.steps, records=True, time_sweeps=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    if rc not in (les.LES_OK, les.LES_WARN_NOT_CONVERGED):
        raise SystemExit(f"les_step failed: {rc}")

    K = p["n_subiter"]
    sweeps_step = st["sweeps_total"] / args.steps
    sw_k0 = float(np.mean([r["sweeps"] for i, r in enumerate(recs) if i % K == 0]))
    sw_k1 = float(np.mean([r["sweeps"] for i, r in enumerate(recs) if i % K != 0])) if K > 1 else 0.0
    ms_step = wall / args.steps * 1e3
    value = ncell * args.steps / wall / 1e6

    avg_sweep = st["sweep_seconds"] / max(st["sweeps_timed"], 1)
    bytes_launch = sweep_bytes_per_cell(p) * ncell
    achieved = bytes_launch / avg_sweep / 1e9
    diag = sim.diagnostics()

    out = {
        "metric": "Mcell-steps/s and Poisson s/step at residual 1e-6, plain guess",
        "value": value,
        "unit": "Mcell-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if p["precision"] == "fp32" else "f64",
        "data": "synthetic",
        "config": {
            "workload": (f"synthetic stratocumulus LES step, {p['nx']}x{p['ny']}x{p['nz']} cells, "
                         f"{p['dx']:g}x{p['dy']:g}x{p['dz']:g} m, dt {p['dt']:g} s, "
                         f"{p['poisson_scheme']} Poisson to rel. residual {p['poisson_tol']:g}, "
                         f"K={K}"),
            "grid": [p["nx"], p["ny"], p["nz"]],
            "precision": p["precision"],
        },
        "poisson_s_per_step": st["poisson_seconds"] / args.steps,
        "sweeps_per_step": sweeps_step,
        "sweeps_per_solve_k0": sw_k0,
        "sweeps_per_solve_k1": sw_k1,
        "not_converged": st["not_converged"],
        "res_rel_max": st["res_rel_max"],
        "cfl": diag["cfl"],
        "roofline": {
            "bound": "hbm",
            "kernel": f"sweep_kernel<{'float' if p['precision'] == 'fp32' else 'double'}, cheb>",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": None,
            "avg_launch_us": avg_sweep * 1e6,
            "bytes_per_launch": bytes_launch,
            "note": ("working set of the sweep is about 134 MB, inside the 256 MB Infinity Cache"
                     if bytes_launch < 256e6 else "working set exceeds the 256 MB Infinity Cache"),
        },
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(p, sweeps_step, args.cpu_crop)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
