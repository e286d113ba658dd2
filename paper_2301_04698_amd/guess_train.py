"""Training and evaluation of the learned Poisson initial guess on the GPU.

Pairs come from the solver itself: runs with the previous-solution guess
dump, every step, the right-hand side and solution of each sub-iteration's
solve; consecutive steps give (base = last step's solution, rhs, phi*)
triples, stored as normalised network inputs and targets (les_cnn_pair).
The three-input network (--inputs 3) learns the first solve of a step from
runs with the extrapolated-pressure guess: (base = alpha0 (p^n - p^{n-1}),
rhs, phi*) of every step's first solve (les_cnn_pair3).
Training draws random crops (les_cnn_gather) and runs the library's own
forward, loss, backward and Adam kernels (les_cnn_train_step).  Every
arithmetic step runs in the HIP library; this module only drives it.

Command line:
    python -m paper_2301_04698_amd.guess_train --workload C4 --out weights.npy
    python -m paper_2301_04698_amd.guess_train --workload C4 --inputs 3 --out weights3.npy
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

import les_inputs as li  # noqa: E402

from . import cnn, les  # noqa: E402

BLOCKS = [(27 * ci * co, 27 * ci, co) for ci, co in zip(cnn.CIN, cnn.COUT)]
BLOCKS3 = [(27 * cnn.cin(l, 3) * co, 27 * cnn.cin(l, 3), co) for l, co in enumerate(cnn.COUT)]
DEFAULT_ALPHA = 0.1


def log(msg):
    print(msg, flush=True)


def collect(p, seeds, windows, window_len, device="cuda"):
    """Training pairs from runs of workload p (one per seed).  windows: step
    indices where a window of window_len + 1 dumped steps starts; each
    window gives window_len x n_subiter pairs.  Returns (X, T) float32
    tensors of shape (npairs, nz, ny, nx)."""
    import torch
    K = p["n_subiter"]
    shape = (p["nz"], p["ny"], p["nx"])
    n = int(np.prod(shape))
    npairs = len(seeds) * len(windows) * window_len * K
    X = torch.empty((npairs,) + shape, dtype=torch.float32, device=device)
    T = torch.empty_like(X)
    q = 0
    for seed in seeds:
        ps = dict(p, seed=int(seed), guess="previous")
        sim = les.LES(ps, li.initial_state(ps), device=device)
        rhs = torch.empty(K * n, dtype=sim.dtype, device=device)
        phi = torch.empty_like(rhs)
        scratch = None
        done = 0
        for w0 in windows:
            if w0 > done:
                sim.step(w0 - done)
                done = w0
            prev = None
            for m in range(window_len + 1):
                sim.step(1, dump=(rhs, phi))
                done += 1
                if prev is not None:
                    for k in range(K):
                        sl = slice(k * n, (k + 1) * n)
                        cnn.pair(sim, rhs[sl], prev[sl], phi[sl], X[q], T[q], scratch)
                        q += 1
                prev = phi.clone()
            log(f"collect: seed {seed} steps {done} pairs {q}/{npairs}")
        sim.close()
    assert q == npairs
    return X, T


def collect3(p, seeds, windows, window_len, device="cuda"):
    """Pairs of the three-input network: each of window_len consecutive
    steps from every window start gives the (inputs, target) of its first
    solve, from runs with the extrapolated guess.  Returns (X, T) float32
    tensors of shapes (npairs, 3, nz, ny, nx) and (npairs, nz, ny, nx)."""
    import torch
    K = p["n_subiter"]
    shape = (p["nz"], p["ny"], p["nx"])
    n = int(np.prod(shape))
    npairs = len(seeds) * len(windows) * window_len
    X = torch.empty((npairs, 3) + shape, dtype=torch.float32, device=device)
    T = torch.empty((npairs,) + shape, dtype=torch.float32, device=device)
    q = 0
    for seed in seeds:
        ps = dict(p, seed=int(seed), guess="extrapolate")
        sim = les.LES(ps, li.initial_state(ps), device=device)
        rhs = torch.empty(K * n, dtype=sim.dtype, device=device)
        phi, base = torch.empty_like(rhs), torch.empty_like(rhs)
        scratch = None
        done = 0
        for w0 in windows:
            if w0 > done:
                sim.step(w0 - done)
                done = w0
            for m in range(window_len):
                sim.step(1, dump=(rhs, phi), dump_base=base)
                done += 1
                cnn.pair3(sim, rhs[:n], base[:n], phi[:n], X[q], T[q], scratch)
                q += 1
            log(f"collect: seed {seed} steps {done} pairs {q}/{npairs}")
        sim.close()
    assert q == npairs
    return X, T


def train(X, T, p, iters=4000, batch=16, crop=32, lr=2e-3, seed=0, alpha=DEFAULT_ALPHA,
          log_every=200, init=None):
    """Adam on random crops with a cosine learning-rate decay.  The loss is
    evaluated on crop x crop interior cells (output crop + 2).  Returns
    (params float32 tensor, loss history [(iteration, loss)])."""
    import torch
    inputs = 1 if X.dim() == 4 else X.shape[1]
    npairs, nz, ny, nx = X.shape[0], X.shape[-3], X.shape[-2], X.shape[-1]
    blocks = BLOCKS if inputs == 1 else BLOCKS3
    p0 = torch.from_numpy(init if init is not None else li.cnn_init(seed, blocks)).float()
    tr = cnn.Trainer(p0, batch, nz, crop + 2, crop + 2, p["dx"], p["dy"], p["dz"], alpha=alpha,
                     lr=lr, device=X.device)
    rng = np.random.default_rng(seed)
    xshape = (batch, nz, crop + 10, crop + 10) if inputs == 1 else \
        (batch, inputs, nz, crop + 10, crop + 10)
    xb = torch.empty(xshape, dtype=torch.float32, device=X.device)
    tb = torch.empty((batch, nz, crop + 2, crop + 2), dtype=torch.float32, device=X.device)
    hist = []
    for it in range(iters):
        tr.hyper = (lr * 0.5 * (1 + math.cos(math.pi * it / iters)),) + tr.hyper[1:]
        crops = np.stack([rng.integers(0, npairs, batch), rng.integers(0, ny, batch),
                          rng.integers(0, nx, batch)], axis=1).astype(np.int32)
        cnn.gather(X, T, torch.from_numpy(crops.reshape(-1)), crop + 2, crop + 2, xb, tb)
        want = it % log_every == 0 or it == iters - 1
        val = tr.step(xb, tb, want_loss=want)
        if want:
            hist.append((it, val))
            log(f"train: iteration {it} loss {val:.5f}")
    return tr.params.detach().clone(), hist


def run_mode(p, state, mode, nsteps, params=None, alpha=DEFAULT_ALPHA, device="cuda", pbar=None,
             passes=1):
    """nsteps timed steps after one untimed step (which fills the history)
    from `state` (p relative to the FP64 profile pbar) with the given guess
    mode (and network passes per solve in the learned form); returns
    per-step figures."""
    import torch
    ps = dict(p, guess=mode, guess_passes=passes if mode == "learned" else 0)
    sim = les.LES(ps, state, device=device, pbar=pbar)
    if mode in ("learned", "learned3"):
        cnn.bind(sim, params, alpha)
    sim.step(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    recs, acc = [], None
    done = 0
    while done < nsteps:
        m = min(50, nsteps - done)
        rc, st_m, r = sim.step(m, records=True)
        recs += r
        if acc is None:
            acc = dict(st_m)
        else:
            for key in ("sweeps_total", "not_converged", "poisson_seconds", "seconds"):
                acc[key] += st_m[key]
            acc["res_rel_max"] = max(acc["res_rel_max"], st_m["res_rel_max"])
        done += m
        log(f"evaluate {mode}: {done}/{nsteps} steps, {acc['sweeps_total'] / done:.0f} sweeps/step")
    st = acc
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    K = p["n_subiter"]
    out = dict(
        mode=mode,
        passes=passes if mode == "learned" else None,
        ms_per_step=wall / nsteps * 1e3,
        mcell_steps_per_s=p["nx"] * p["ny"] * p["nz"] * nsteps / wall / 1e6,
        poisson_s_per_step=st["poisson_seconds"] / nsteps,
        sweeps_per_step=st["sweeps_total"] / nsteps,
        sweeps_per_solve=[float(np.mean([r["sweeps"] for i, r in enumerate(recs) if i % K == k]))
                          for k in range(K)],
        not_converged=st["not_converged"],
        res_rel_max=st["res_rel_max"],
        starts={name: sum(1 for r in recs if r["guess"] == code)
                for code, name in ((0, "zero"), (1, "guess_kept"), (2, "guess_rejected"),
                                   (3, "repeated_from_zero"))},
    )
    sim.close()
    return out


def evaluate(p, params, seed, spinup, nsteps, alpha=DEFAULT_ALPHA, modes=("zero", "previous",
                                                                             "learned"),
             device="cuda", passes=(1,)):
    """Spin up a held-out run with the plain solver, then run each guess
    mode from the same state (the learned form once per pass count; keys
    "learned", "learned_2passes", ...)."""
    ps = dict(p, seed=int(seed), guess="zero")
    sim = les.LES(ps, li.initial_state(ps), device=device)
    done = 0
    while done < spinup:
        m = min(50, spinup - done)
        sim.step(m)
        done += m
        log(f"evaluate: spin-up {done}/{spinup}")
    state, pbar = sim.state_split()
    sim.close()
    res = {}
    for mode in modes:
        for np_ in (passes if mode == "learned" else (1,)):
            key = mode if np_ == 1 else f"{mode}_{np_}passes"
            res[key] = run_mode(ps, state, mode, nsteps, params, alpha, device, pbar=pbar,
                                passes=np_)
            log(f"evaluate: {json.dumps(res[key])}")
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="C4")
    ap.add_argument("--inputs", type=int, default=1, choices=(1, 3),
                    help="1: residual input, every solve; 3: previous pressures and the "
                         "divergence, first solve of a step")
    ap.add_argument("--seeds", default="1000,1001,1002")
    ap.add_argument("--windows", default="40,150,300")
    ap.add_argument("--window-len", type=int, default=3)
    ap.add_argument("--iters", type=int, default=4000)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--crop", type=int, default=32)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--alpha", type=float, default=DEFAULT_ALPHA)
    ap.add_argument("--eval-seed", type=int, default=2000)
    ap.add_argument("--eval-spinup", type=int, default=300)
    ap.add_argument("--eval-steps", type=int, default=40)
    ap.add_argument("--out", required=True,
                    help="weights file to write (or, with --eval-only, to evaluate)")
    ap.add_argument("--passes", default="1",
                    help="network passes per solve evaluated for the one-input network "
                         "(comma list)")
    ap.add_argument("--eval-only", action="store_true",
                    help="evaluate the weights in --out on the held-out run; write <out>.eval.json")
    ap.add_argument("--no-eval", action="store_true")
    a = ap.parse_args()
    import torch
    torch.cuda.set_device(0)
    p = li.workload(a.workload)
    passes = tuple(int(x) for x in a.passes.split(","))
    modes = ("zero", "previous", "learned") if a.inputs == 1 else ("zero", "extrapolate",
                                                                   "learned3")
    if a.eval_only:
        params = torch.from_numpy(np.load(a.out)).cuda()
        t0 = time.perf_counter()
        res = evaluate(p, params, a.eval_seed, a.eval_spinup, a.eval_steps, a.alpha, modes,
                       passes=passes)
        summary = dict(workload=a.workload, weights=os.path.basename(a.out), eval_seed=a.eval_seed,
                       eval_spinup=a.eval_spinup, eval_steps=a.eval_steps,
                       eval_s=time.perf_counter() - t0, eval=res)
        with open(os.path.splitext(a.out)[0] + ".eval.json", "w") as f:
            json.dump(summary, f, indent=1)
        log(json.dumps(summary))
        return
    t0 = time.perf_counter()
    gather_pairs = collect if a.inputs == 1 else collect3
    X, T = gather_pairs(p, [int(s) for s in a.seeds.split(",")],
                        [int(w) for w in a.windows.split(",")], a.window_len)
    t1 = time.perf_counter()
    params, hist = train(X, T, p, a.iters, a.batch, a.crop, a.lr, alpha=a.alpha)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    del X, T
    np.save(a.out, params.cpu().numpy().astype(np.float32))
    res = None if a.no_eval else evaluate(p, params, a.eval_seed, a.eval_spinup, a.eval_steps,
                                          a.alpha, modes, passes=passes)
    npairs = len(a.seeds.split(",")) * len(a.windows.split(",")) * a.window_len * \
        (p["n_subiter"] if a.inputs == 1 else 1)
    summary = dict(command="python -m paper_2301_04698_amd.guess_train " + " ".join(sys.argv[1:]),
                   workload=a.workload, inputs=a.inputs,
                   seeds=[int(x) for x in a.seeds.split(",")],
                   windows=[int(x) for x in a.windows.split(",")], window_len=a.window_len,
                   pairs=npairs, crop_samples=a.iters * a.batch, collect_s=t1 - t0,
                   train_s=t2 - t1, loss=hist, alpha=a.alpha, iters=a.iters, batch=a.batch,
                   crop=a.crop, lr=a.lr, schedule="cosine", eval=res)
    with open(os.path.splitext(a.out)[0] + ".json", "w") as f:
        json.dump(summary, f, indent=1)
    log(json.dumps(summary))


if __name__ == "__main__":
    main()
