"""The training-pair entry point that allocates nothing
(les_cnn_pair_noalloc, include/les_cnn.h) against les_cnn_pair, which takes
a caller scratch buffer: two calls in a row on one GPU, the second on a
smaller grid of the other precision (its fixed device scratch then holds the
first call's partial sums), each equal to les_cnn_pair bit for bit, and the
pair itself checked against the oracle's Laplacian."""
import numpy as np
import pytest

import les_inputs as li

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2301_04698_amd import cnn, les
    les.load()
    cnn.lib()
    return cnn


def _case(gpu, oracle_lib, nx, ny, nz, precision, seed):
    import torch
    from paper_2301_04698_amd import les
    print(f"no-alloc pair: {nx}x{ny}x{nz} {precision} seed {seed}", flush=True)
    p = li.workload("C1", nx=nx, ny=ny, nz=nz, precision=precision)
    sim = les.LES(p)
    shape = (nz, ny, nx)
    dt = torch.float32 if precision == "fp32" else torch.float64
    rhs = li.random_field(shape, seed=seed)
    base = li.random_field(shape, seed=seed + 1) * 50.0
    phi = base + li.random_field(shape, seed=seed + 2) * 5.0
    cast = lambda a: torch.from_numpy(a).to(device="cuda", dtype=dt).contiguous()
    R, B, P = cast(rhs), cast(base), cast(phi)
    x0, t0 = (torch.full(shape, 7.0, device="cuda") for _ in range(2))
    x1, t1 = (torch.full(shape, -3.0, device="cuda") for _ in range(2))
    s0 = gpu.pair(sim, R, B, P, x0, t0)
    s1 = gpu.pair_noalloc(sim, R, B, P, x1, t1)
    torch.cuda.synchronize()
    assert s1 == s0
    assert torch.equal(x1, x0) and torch.equal(t1, t0)
    # the pair itself: r = rhs - L base in FP64 on the stored values
    bq = B.double().cpu().numpy()
    r = R.double().cpu().numpy() - oracle_lib.laplacian(p, bq)
    s_ref = np.sqrt(np.mean(r ** 2))
    assert s1 == pytest.approx(s_ref, rel=1e-6)
    xr = x1.double().cpu().numpy()
    assert np.linalg.norm(xr - r / s_ref) <= 1e-6 * np.linalg.norm(r / s_ref)
    sim.close()


def test_no_alloc_pair_matches_scratch_pair_twice(gpu, oracle_lib):
    _case(gpu, oracle_lib, 72, 40, 36, "fp32", 31)
    _case(gpu, oracle_lib, 20, 12, 8, "fp64", 41)
