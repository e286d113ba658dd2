"""The trained guess network against the method without it: train on pairs
the solver generates on one seed, evaluate on a held-out seed, and require
fewer sweeps and fewer Poisson seconds per step than both the plain
(zero-guess) solve and the uncorrected previous-solution guess, at the same
residual tolerance."""
import numpy as np
import pytest

import les_inputs as li

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def trained():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2301_04698_amd import guess_train as gt
    p = li.workload("C3s")
    X, T = gt.collect(p, [1000], windows=[12], window_len=6)
    params, hist = gt.train(X, T, p, iters=300, batch=8, crop=24, lr=2e-3, log_every=50)
    return p, params, hist


def test_training_reduces_loss(trained):
    p, params, hist = trained
    first, last = hist[0][1], hist[-1][1]
    print("loss history", hist)
    assert last < 0.3 * first and last < 0.2, hist


def test_trained_guess_saves_sweeps_and_time(trained):
    from paper_2301_04698_amd import guess_train as gt
    p, params, _ = trained
    res = gt.evaluate(p, params, seed=2000, spinup=20, nsteps=8)
    for mode, r in res.items():
        print(mode, r)
        assert r["not_converged"] == 0 and r["res_rel_max"] <= p["poisson_tol"]
    z, prev, learned = res["zero"], res["previous"], res["learned"]
    assert learned["sweeps_per_step"] < 0.85 * z["sweeps_per_step"]
    assert learned["sweeps_per_step"] < prev["sweeps_per_step"]
    assert learned["poisson_s_per_step"] < z["poisson_s_per_step"]
