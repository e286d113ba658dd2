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
FP64 CPU oracle timed on the host on a bounded sample.  `value` is the plain
form (every solve starts from zero).  The learned form (each solve starts
from the previous step's solution corrected by the trained guess network,
whose inference time counts in the Poisson seconds) runs the same steps
from the same initial state and is reported under "learned".  The largest
single-GPU domain, 1024 x 1024 x 256, is reported under "c5": both forms'
Mcell-steps/s, Poisson seconds and sweeps per step from one state after a
few warm-up steps, and the streamed sweep's HBM GB/s.
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
CASE_LABEL = {"cloud_layer": "synthetic stratocumulus",
              "bubble": "dry bubble (density current / rising bubble)"}

# HBM bytes per launch of the one-sweep Chebyshev kernel measured with
# rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE (FETCH scaled x2.0, WRITE x1.0 by a
# 1 GiB copy calibration); see profiles/sweep_kernel_hbm_traffic_pmc.md.
# Valid only for the sweep source it was taken on (sha256 prefix).
SWEEP_SOURCE = os.path.join(ROOT, "paper_2301_04698_amd", "csrc", "k_tsweep.hip")
GUESS_WEIGHTS = os.path.join(ROOT, "paper_2301_04698_amd", "weights", "guess_256x256x128.npy")
MEASURED_TRAFFIC = {
    "sha256": "013a1b1cb19709d2",
    "bytes": {(256, 256, 128): 104_610_944 + 33_554_432, (512, 512, 256): 841_642_816 + 268_435_456},
}

def measured_traffic(p, S):
    import hashlib
    if S != 1:
        return None
    with open(SWEEP_SOURCE, "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()[:16]
    if sha != MEASURED_TRAFFIC["sha256"]:
        return None
    return MEASURED_TRAFFIC["bytes"].get((p["nx"], p["ny"], p["nz"]))


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="C2")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--oracle-timings", action="store_true",
                    help="only time the oracle on the host (the benchmark runs this in a child "
                         "process) and print one JSON line")
    ap.add_argument("--cpu-crop", type=int, default=128,
                    help="horizontal size of the crop the oracle's non-Poisson work is timed on")
    ap.add_argument("--mode", choices=("step", "sweeps", "copy"), default="step",
                    help="step: the LES step benchmark; sweeps: a fixed number of Poisson "
                         "sweeps on the workload's grid; copy: a device-to-device copy of "
                         "--bytes bytes (calibrates the HBM byte counters)")
    ap.add_argument("--sweeps", type=int, default=200)
    ap.add_argument("--sweeps-per-launch", type=int, default=0)
    ap.add_argument("--bytes", type=int, default=1 << 30)
    ap.add_argument("--guess-weights", default=GUESS_WEIGHTS,
                    help="trained guess network for the learned form ('' to skip it)")
    ap.add_argument("--guess-alpha", type=float, default=0.1)
    ap.add_argument("--guess-passes", type=int, default=2,
                    help="network passes per guessed solve in the learned form (each pass "
                         "after the first corrects the last one's guess from its residual)")
    ap.add_argument("--c5-warmup", type=int, default=3,
                    help="largest-domain leg (1024x1024x256): untimed steps from the initial "
                         "state (learned form; its first step starts from zero)")
    ap.add_argument("--c5-steps", type=int, default=5,
                    help="largest-domain leg: timed steps of each form from the same state "
                         "(0 skips the leg)")
    ap.add_argument("--advection", choices=("quick", "weno3"), default="quick",
                    help="face-value scheme of the advection (QUICK, or third-order WENO with a "
                         "Lax-Friedrichs flux)")
    return ap.parse_args()


def run_sweeps(args):
    """Fixed-count Poisson solve on a seeded right-hand side of the
    workload's grid; per-sweep time from HIP events around the solve."""
    import numpy as np
    import torch

    import les_inputs as li
    from paper_2301_04698_amd import les

    p = li.workload(args.workload, sweeps_per_launch=args.sweeps_per_launch)
    shape = (p["nz"], p["ny"], p["nx"])
    n = p["nx"] * p["ny"] * p["nz"]
    sim = les.LES(p, device="cuda:0")
    dt = torch.float32 if p["precision"] == "fp32" else torch.float64
    rhs = torch.from_numpy(li.random_field(shape, seed=3)).to("cuda:0", dt)
    sim.poisson_solve(rhs, fixed_sweeps=10)
    _, st, _ = sim.poisson_solve(rhs, fixed_sweeps=args.sweeps)
    per = st["seconds"] / args.sweeps
    bpc = sweep_bytes_per_cell(p)
    print(json.dumps({
        "mode": "sweeps", "workload": args.workload, "grid": [p["nx"], p["ny"], p["nz"]],
        "precision": p["precision"], "scheme": p["poisson_scheme"], "sweeps": args.sweeps,
        "us_per_sweep": per * 1e6, "bytes_per_sweep": bpc * n,
        "algorithmic_GBs": bpc * n / per / 1e9, "frac_of_8TBs": bpc * n / per / 1e9 / HBM_PEAK_GBS,
        "note": "solve time includes rhs centring and the final residual check"}), flush=True)


def run_copy(args):
    import torch
    n = args.bytes // 4
    a = torch.ones(n, device="cuda:0", dtype=torch.float32)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 10
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    s = e0.elapsed_time(e1) / 1e3 / reps
    print(json.dumps({"mode": "copy", "bytes_read": 4 * n, "bytes_written": 4 * n,
                      "us_per_copy": s * 1e6, "GBs_read_plus_write": 8 * n / s / 1e9}), flush=True)


def sweep_kernel_name(p, S):
    """Template instance of the plain (no residual check) sweep launch."""
    es = 8 if p["precision"] == "fp64" else 4
    cheb = "true" if p["poisson_scheme"] == "chebyshev" else "false"
    T = "double" if es == 8 else "float"
    if S != 1:
        return f"sweep2_kernel<{T}, 4, {cheb}, false>"
    streamed = 4.0 * p["nx"] * p["ny"] * p["nz"] * es > 192e6
    if p["nx"] >= 256 and p["ny"] >= 4:
        wx, ty = 4, (4 if streamed else 2)
    else:
        wx, ty = 1, (16 if streamed else 4)
        if p["ny"] < ty:
            ty = 1 if p["ny"] < 4 else 4
    return f"sweep1_kernel<{T}, {wx}, {ty}, {cheb}, false, {'true' if streamed else 'false'}>"


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
    pc["nx"], pc["ny"] = min(crop, p["nx"]), min(crop, p["ny"])
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


def oracle_timings():
    """The oracle (serial FP64 C, one thread) timed on the host: all ten steps
    of the 32^3 workload, one step of the 64^3 companion of the 512x512x256
    workload, and the per-sweep cell-update rate of its Poisson sweep at the
    size of every workload (the difference of a 3-sweep and a 1-sweep solve,
    so the per-solve setup cancels).  Runs in a child process that never
    touches the GPU; prints one JSON line."""
    import les_inputs as li
    import oracle
    out = {}
    p = li.workload("C1")
    st = li.initial_state(p)
    t0 = time.perf_counter()
    recs, _ = oracle.step(p, st, nsteps=10)
    t = time.perf_counter() - t0
    out["c1_ten_steps"] = {"seconds": t, "sweeps": sum(r["sweeps"] for r in recs),
                           "mcell_steps_per_s": p["nx"] * p["ny"] * p["nz"] * 10 / t / 1e6}
    p = li.workload("C3s")
    st = li.initial_state(p)
    t0 = time.perf_counter()
    recs, _ = oracle.step(p, st, nsteps=1)
    t = time.perf_counter() - t0
    out["c3_companion_64cubed_step"] = {"seconds": t, "sweeps": sum(r["sweeps"] for r in recs),
                                        "mcell_steps_per_s": 64 ** 3 / t / 1e6}
    # per-sweep rate: (t(1 + m sweeps) - t(1 sweep)) / m; a sweep's cost does
    # not depend on the values, so the large grids take one seeded plane
    # repeated over the levels; sizes beyond the time budget are skipped
    import numpy as np
    rates = {}
    t_start = time.perf_counter()
    for name, m in (("C1", 200), ("C2", 10), ("C3", 4), ("C5", 2)):
        p = li.workload(name)
        key = f"{p['nx']}x{p['ny']}x{p['nz']}"
        if time.perf_counter() - t_start > 150:
            rates[key] = "skipped (time budget)"
            continue
        plane = li.random_field((1, p["ny"], p["nx"]), seed=3)
        rhs = np.ascontiguousarray(np.broadcast_to(plane, (p["nz"], p["ny"], p["nx"])))
        ts = []
        for nsw in (1, 1 + m):
            t0 = time.perf_counter()
            oracle.poisson(p, rhs, fixed_sweeps=nsw)
            ts.append(time.perf_counter() - t0)
        per = (ts[1] - ts[0]) / m
        rates[key] = {"s_per_sweep": per, "sweeps_timed": m, "one_sweep_solve_s": ts[0],
                      "mcell_updates_per_s": rhs.size / per / 1e6 if per > 0 else None}
        del rhs
    out["sweep_rates"] = rates
    print(json.dumps(out), flush=True)


def host_cpu():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "nproc": len(os.sched_getaffinity(0)), "cpu_count": os.cpu_count()}


def learned_form(p, args, plain_sweeps, plain_poisson, plain_value):
    """The same steps from the same initial state with the learned guess."""
    import numpy as np
    import torch

    import les_inputs as li
    from paper_2301_04698_amd import cnn, les

    pl = dict(p, guess="learned", guess_passes=args.guess_passes)
    sim = les.LES(pl, li.initial_state(pl), device="cuda:0")
    cnn.bind(sim, torch.from_numpy(np.load(args.guess_weights)), args.guess_alpha)
    if args.warmup > 0:
        sim.step(args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc, st, recs = sim.step(args.steps, records=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    if rc not in (les.LES_OK, les.LES_WARN_NOT_CONVERGED):
        raise SystemExit(f"les_step (learned guess) failed: {rc}")
    K = p["n_subiter"]
    sweeps = st["sweeps_total"] / args.steps
    poisson = st["poisson_seconds"] / args.steps
    value = p["nx"] * p["ny"] * p["nz"] * args.steps / wall / 1e6
    sim.close()
    return {
        "value": value,
        "unit": "Mcell-steps/s",
        "ms_per_step": wall / args.steps * 1e3,
        "poisson_s_per_step": poisson,
        "sweeps_per_step": sweeps,
        "sweeps_per_solve": [float(np.mean([r["sweeps"] for i, r in enumerate(recs) if i % K == k]))
                             for k in range(K)],
        "iterations_saved_per_step": plain_sweeps - sweeps,
        "poisson_speedup": plain_poisson / poisson,
        "speedup": value / plain_value,
        "not_converged": st["not_converged"],
        "res_rel_max": st["res_rel_max"],
        "weights": os.path.relpath(args.guess_weights, ROOT),
        "guess_passes": args.guess_passes,
        "note": ("each solve after the first step starts from the previous step's solution of the "
                 "same sub-iteration plus the network's correction (guess_passes passes, each "
                 "after the first correcting the last one's guess from its residual); the "
                 "network's inference time is inside poisson_s_per_step; same residual test as "
                 "the plain form"),
    }


def progress(msg):
    """Progress of a long run on stderr (the JSON line stays alone on stdout)."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def largest_domain(args):
    """The largest single-GPU domain, 1024 x 1024 x 256 (268 M cells, FP32,
    the sweep's arrays far beyond the Infinity Cache): args.c5_warmup
    untimed steps from the initial state with the learned form (the first
    of them starts every solve from zero), then args.c5_steps timed steps of
    the learned form and, from the same state (fields and the FP64 pressure
    profile copied on the device), of the plain form."""
    import numpy as np
    import torch

    import les_inputs as li
    from paper_2301_04698_amd import cnn, les

    p = li.workload("C5")
    ncell = p["nx"] * p["ny"] * p["nz"]
    K = p["n_subiter"]
    T = args.c5_steps
    prm = torch.from_numpy(np.load(args.guess_weights))

    def timed(sim):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, st, recs = sim.step(T, records=True, time_sweeps=True)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        if rc not in (les.LES_OK, les.LES_WARN_NOT_CONVERGED):
            raise SystemExit(f"les_step (1024x1024x256) failed: {rc}")
        return {
            "value": ncell * T / wall / 1e6,
            "unit": "Mcell-steps/s",
            "ms_per_step": wall / T * 1e3,
            "poisson_s_per_step": st["poisson_seconds"] / T,
            "sweeps_per_step": st["sweeps_total"] / T,
            "sweeps_per_solve": [r["sweeps"] for r in recs],
            "starts": [r["guess"] for r in recs],
            "not_converged": st["not_converged"],
            "res_rel_max": st["res_rel_max"],
        }, st

    t0 = time.perf_counter()
    sim = les.LES(dict(p, guess="learned", guess_passes=args.guess_passes), li.initial_state(p),
                  device="cuda:0")
    cnn.bind(sim, prm, args.guess_alpha)
    t_init = time.perf_counter() - t0
    progress(f"1024x1024x256: set up in {t_init:.0f} s")
    t0 = time.perf_counter()
    for w in range(args.c5_warmup):
        _, st, recs = sim.step(1, records=True)
        progress(f"1024x1024x256: warm-up step {w + 1}/{args.c5_warmup}, "
                 f"{st['sweeps_total']} sweeps, {st['seconds']:.1f} s, solves "
                 f"{[(r['sweeps'], r['guess']) for r in recs]}")
    torch.cuda.synchronize()
    t_warm = time.perf_counter() - t0
    snap = {k: v.clone() for k, v in sim.fields.items()}
    _, pbar = sim.pressure()
    learned, _ = timed(sim)
    progress(f"1024x1024x256: learned form {learned['ms_per_step'] / 1e3:.1f} s/step, solves "
             f"{learned['sweeps_per_solve']} sweeps, starts {learned['starts']}")
    sim.close()
    del sim
    torch.cuda.empty_cache()
    sim = les.LES(p, snap, device="cuda:0", pbar=pbar)
    del snap
    plain, st = timed(sim)
    progress(f"1024x1024x256: plain form {plain['ms_per_step'] / 1e3:.1f} s/step, solves "
             f"{plain['sweeps_per_solve']} sweeps")
    sim.close()
    del sim
    torch.cuda.empty_cache()
    S = 1
    avg = st["sweep_seconds"] / max(st["sweeps_timed"], 1)
    bytes_launch = sweep_bytes_per_cell(p) * ncell
    achieved = bytes_launch / avg / 1e9
    learned["guess_passes"] = args.guess_passes
    learned["speedup"] = learned["value"] / plain["value"]
    learned["poisson_speedup"] = plain["poisson_s_per_step"] / learned["poisson_s_per_step"]
    learned["iterations_saved_per_step"] = plain["sweeps_per_step"] - learned["sweeps_per_step"]
    return {
        "workload": (f"synthetic stratocumulus LES step, {p['nx']}x{p['ny']}x{p['nz']} cells, "
                     f"{p['dx']:g}x{p['dy']:g}x{p['dz']:g} m, dt {p['dt']:g} s, "
                     f"{p['poisson_scheme']} Poisson to rel. residual {p['poisson_tol']:g}, K={K}"),
        "grid": [p["nx"], p["ny"], p["nz"]],
        "warmup": args.c5_warmup,
        "steps": T,
        "note": (f"{args.c5_warmup} untimed steps from the initial state (learned form, first "
                 f"step from zero; {t_warm:.0f} s), then {T} timed step(s) of each form from that "
                 f"state; setup {t_init:.0f} s"),
        "plain": plain,
        "learned": learned,
        "sweep": {
            "bound": "hbm",
            "kernel": sweep_kernel_name(p, S),
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "avg_launch_us": avg * 1e6,
            "bytes_per_launch": bytes_launch,
            "note": ("plain sweeps between residual checks, HIP events on the library's stream; "
                     "arrays of 4.3 GB per sweep, beyond the 256 MB Infinity Cache"),
        },
    }


def main():
    args = parse()
    if args.oracle_timings:
        return oracle_timings()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the library's LES step runs on a single "
              "MI355X and has no multi-GPU decomposition; use --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    # The oracle's own timings run on the host beside the GPU legs, started
    # before anything initialises the GPU (a child of a GPU process must not
    # exec).
    timings = None
    if not args.no_cpu_baseline and args.mode == "step":
        import subprocess
        timings = subprocess.Popen([sys.executable, os.path.abspath(__file__), "--oracle-timings"],
                                   stdout=subprocess.PIPE, text=True)

    import numpy as np
    import torch

    import les_inputs as li
    from paper_2301_04698_amd import les

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.mode == "sweeps":
        return run_sweeps(args)
    if args.mode == "copy":
        return run_copy(args)
    p = li.workload(args.workload, sweeps_per_launch=args.sweeps_per_launch,
                    advection=args.advection)
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

    S = sim.cfg.sweeps_per_launch or 1
    avg_sweep = st["sweep_seconds"] / max(st["sweeps_timed"], 1)
    avg_launch = avg_sweep * S
    es = 4 if p["precision"] == "fp32" else 8
    # one sweep: sweep_bytes_per_cell; two fused sweeps: 3 arrays in, 2 out
    bytes_launch = (sweep_bytes_per_cell(p) if S == 1 else 5 * es) * ncell
    achieved = bytes_launch / avg_launch / 1e9
    diag = sim.diagnostics()

    out = {
        "metric": "Mcell-steps/s and Poisson s/step at residual 1e-6, plain vs learned guess",
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
            "workload": (f"{CASE_LABEL.get(p['init'], p['init'])} LES step, "
                         f"{p['nx']}x{p['ny']}x{p['nz']} cells, "
                         f"{p['dx']:g}x{p['dy']:g}x{p['dz']:g} m, dt {p['dt']:g} s, "
                         f"{p['poisson_scheme']} Poisson to rel. residual {p['poisson_tol']:g}, "
                         f"K={K}, {p['advection']} advection"),
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
            "kernel": sweep_kernel_name(p, S),
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": measured_traffic(p, sim.cfg.sweeps_per_launch or 1),
            "avg_launch_us": avg_launch * 1e6,
            "sweeps_per_launch": S,
            "bytes_per_launch": bytes_launch,
            "note": (f"working set of the sweep {bytes_launch / 1e6:.0f} MB, "
                     + ("inside" if bytes_launch < 256e6 else "beyond")
                     + " the 256 MB Infinity Cache"),
        },
    }
    progress(f"{p['nx']}x{p['ny']}x{p['nz']}: plain form {value:.1f} Mcell-steps/s")
    if p["init"] != "cloud_layer":
        out["learned"] = None  # the guess network was trained on the cloud-layer workload
    elif args.guess_weights and os.path.exists(args.guess_weights):
        out["learned"] = learned_form(p, args, sweeps_step, st["poisson_seconds"] / args.steps,
                                      value)
    else:
        out["learned"] = None
    sim.close()
    del sim
    torch.cuda.empty_cache()
    if (args.c5_steps > 0 and args.workload == "C2" and args.guess_weights
            and os.path.exists(args.guess_weights)):
        out["c5"] = largest_domain(args)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(p, sweeps_step, args.cpu_crop)
        out["cpu_baseline"]["host"] = host_cpu()
        if timings is not None:
            try:
                so, _ = timings.communicate(timeout=300)
                out["cpu_baseline"]["oracle_timings"] = json.loads(so.strip().splitlines()[-1])
            except Exception as e:  # report, never fail the benchmark for it
                timings.kill()
                out["cpu_baseline"]["oracle_timings"] = {"error": repr(e)}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
