"""Precision study of the 512 x 512 x 256 workload: FP32 storage and stencils
with FP64 reductions and saturation adjustment, against the full-FP64 GPU
path at full size and against the FP64 oracle on the 64^3 companion run
(same spacing, profile and forcing).  Both comparisons apply identical
sweep counts on both sides, so the differences are those of precision,
not of where a solve stopped.  Per-field relative L2 errors are printed.
"""
import numpy as np
import pytest

import les_inputs as li

pytestmark = pytest.mark.gpu

FIELDS = ("u", "v", "w", "thl", "qt", "p")


@pytest.fixture(scope="module")
def les():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2301_04698_amd import les
    les.load()
    return les


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def f32(st):
    return {k: v.astype(np.float32).astype(np.float64) for k, v in st.items()}


def test_companion_64cubed_fp32_per_step(les, oracle_lib):
    """Five steps of the 64^3 companion: each step starts both sides from
    the oracle's state (rounded to FP32) and the GPU replays the oracle's
    sweep counts; per-step error per field <= 1e-5."""
    p = li.workload("C3s")
    st = li.initial_state(p)
    rng = np.random.default_rng(31)
    for k in ("u", "v", "w"):
        st[k] = st[k] + 0.2 * rng.standard_normal(st[k].shape)
    st = f32(st)
    worst = {k: 0.0 for k in FIELDS}
    for n in range(5):
        ost = {k: v.copy() for k, v in st.items()}
        recs, _ = oracle_lib.step(p, ost, nsteps=1)
        sim = les.LES(p, st)
        sim.step(1, replay=[r["sweeps"] for r in recs])
        gst = sim.state_numpy()
        errs = {k: rel(gst[k], ost[k]) for k in FIELDS}
        print(f"step {n}: sweeps {[r['sweeps'] for r in recs]} per-field rel L2 "
              + " ".join(f"{k} {e:.2e}" for k, e in errs.items()))
        for k, e in errs.items():
            worst[k] = max(worst[k], e)
        st = f32(ost)
    for k, e in worst.items():
        assert e <= 1e-5, (k, e)


def test_full_size_fp32_against_fp64_gpu(les):
    """512 x 512 x 256, three steps with 300 sweeps per solve on both paths
    (both beyond the Infinity Cache: the streamed sweep kernel)."""
    p64 = li.workload("C3", precision="fp64")
    p32 = li.workload("C3")
    st = f32(li.initial_state(p32))
    replay = [300] * (3 * p32["n_subiter"])
    s64 = les.LES(p64, st)
    s64.step(3, replay=replay)
    g64 = s64.state_numpy()
    s64.close()
    s32 = les.LES(p32, st)
    s32.step(3, replay=replay)
    g32 = s32.state_numpy()
    errs = {k: rel(g32[k], g64[k]) for k in FIELDS}
    print("512x512x256 after 3 steps, FP32 vs FP64 GPU: "
          + " ".join(f"{k} {e:.2e}" for k, e in errs.items()))
    for k, e in errs.items():
        assert e <= 3e-5, (k, e)
