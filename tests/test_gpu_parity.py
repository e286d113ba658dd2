"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle on
identical seeded inputs.

Bars: FP64 GPU path <= 1e-11 relative L2 per field; FP32 path <= 1e-5
relative L2 per field per step.  For full steps the GPU replays the oracle's
per-solve sweep counts so a stopping decision on the tolerance boundary
cannot shift one side by a check interval.
"""
import numpy as np
import pytest

import les_inputs as li
from conftest import assert_fp32, fmt_fp32, fp32_errors

pytestmark = pytest.mark.gpu

FIELDS = ("u", "v", "w", "thl", "qt", "p")


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2301_04698_amd import les
    les.load()
    return les


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def rel_anom(a, b):
    """Error relative to the deviation of b from its horizontal mean."""
    d = b - b.mean(axis=(1, 2), keepdims=True)
    nd = np.linalg.norm(d)
    return np.linalg.norm(a - b) / (nd if nd > 0 else 1.0)


def _fp32_bars(ost, gst):
    """FP32 bars of one compared step (relative L2 and relative to the
    horizontal anomaly, conftest.assert_fp32)."""
    errs = fp32_errors(gst, ost, FIELDS)
    print("FP32 per-field error (relative / relative to anomaly): " + fmt_fp32(errs))
    assert_fp32(errs)


def with_velocity_noise(p, st, amp, seed):
    rng = np.random.default_rng(seed)
    for k in ("u", "v", "w"):
        st[k] = st[k] + amp * rng.standard_normal(st[k].shape)
    return st


# ------------------------------------------------------------ Poisson

@pytest.mark.parametrize("shape,scheme", [((8, 8, 8), "jacobi"), ((10, 12, 16), "jacobi"),
                                          ((8, 8, 8), "chebyshev"), ((10, 12, 16), "chebyshev"),
                                          ((20, 36, 70), "chebyshev")])
def test_poisson_fp64_matches_oracle(gpu, oracle_lib, shape, scheme):
    import torch
    nz, ny, nx = shape
    p = li.workload("C1", nx=nx, ny=ny, nz=nz, dx=40.0, dy=30.0, dz=10.0, poisson_tol=1e-10,
                    poisson_scheme=scheme)
    rhs = li.random_field(shape, seed=21) + 0.3  # nonzero mean: removed by both sides
    phi_o, st_o = oracle_lib.poisson(p, rhs)
    sim = gpu.LES(p)
    phi_g, st_g, rc = sim.poisson_solve(torch.from_numpy(rhs))
    assert rc == 0 and st_g["status"] == 0 and st_o["status"] == 0
    assert st_g["sweeps"] == st_o["sweeps"]
    assert st_g["res_norm"] <= 1e-10 * st_g["rhs_norm"]
    assert st_g["rhs_norm"] == pytest.approx(st_o["rhs_norm"], rel=1e-13)
    e = rel(phi_g.cpu().numpy(), phi_o)
    assert e <= 1e-11, e


@pytest.mark.parametrize("shape", [(8, 1, 2), (8, 3, 2), (6, 2, 3), (5, 1, 65), (4, 3, 129),
                                   (6, 5, 300)])
def test_poisson_degenerate_grids_match_oracle(gpu, oracle_lib, shape):
    """The smallest grids the library accepts and rows that end one cell into
    a wavefront: nx = 2, 3 (every lane but the first one or two idle, both
    end lanes load their x neighbours), ny = 1..3 (one-row tiles), nx = 65
    and 129 (a second or third wavefront holding a single cell), nx = 300 (a
    256-wide tile whose second wave is ragged and whose others lie beyond
    nx, with a partial tile row in y)."""
    import torch
    nz, ny, nx = shape
    p = li.workload("C1", nx=nx, ny=ny, nz=nz, dx=40.0, dy=30.0, dz=10.0, poisson_tol=1e-10,
                    poisson_scheme="chebyshev")
    rhs = li.random_field(shape, seed=22)
    phi_o, st_o = oracle_lib.poisson(p, rhs)
    sim = gpu.LES(p)
    phi_g, st_g, rc = sim.poisson_solve(torch.from_numpy(rhs), fixed_sweeps=st_o["sweeps"])
    assert st_g["sweeps"] == st_o["sweeps"] and st_o["status"] == 0
    e = rel(phi_g.cpu().numpy(), phi_o)
    assert e <= 1e-11, e


@pytest.mark.parametrize("mean_mode", ["exact", "level", "swept"])
@pytest.mark.parametrize("shape", [(12, 9, 15), (33, 1, 7), (10, 14, 2)])
def test_poisson_mean_modes_match_oracle(gpu, oracle_lib, shape, mean_mode):
    """Every split of the uniform parts (none, the horizontally uniform part
    exact, both uniform parts exact) at odd and degenerate horizontal sizes
    (transforms over 15 x 9, 7 x 1 and 2 x 14 points): the same sweep count
    as the oracle and the same solution.  The right-hand side carries large
    uniform parts of both kinds."""
    import torch
    nz, ny, nx = shape
    p = li.workload("C1", nx=nx, ny=ny, nz=nz, dx=40.0, dy=30.0, dz=10.0, poisson_tol=1e-10,
                    poisson_scheme="chebyshev", mean_mode=mean_mode)
    rng = np.random.default_rng(25)
    rhs = (li.random_field(shape, seed=25) + 3.0 * rng.standard_normal((nz, 1, 1))
           + 2.0 * rng.standard_normal((1, ny, nx)))
    phi_o, st_o = oracle_lib.poisson(p, rhs)
    sim = gpu.LES(p)
    phi_g, st_g, rc = sim.poisson_solve(torch.from_numpy(rhs))
    print(f"{mean_mode} {shape}: {st_o['sweeps']} sweeps", flush=True)
    assert rc == 0 and st_o["status"] == 0 and st_g["status"] == 0
    assert st_g["sweeps"] == st_o["sweeps"]
    assert st_g["res_norm"] <= 1e-10 * st_g["rhs_norm"]
    assert rel(phi_g.cpu().numpy(), phi_o) <= 1e-11
    sim.close()


@pytest.mark.parametrize("every,spl", [(1, 1), (3, 1), (1, 2), (4, 2), (25, 2)])
def test_poisson_check_intervals_match_oracle(gpu, oracle_lib, every, spl):
    """Residual checks every 1, 3, 4 or 25 sweeps with one- and two-sweep
    launches: a check is decided inside the next one-sweep launch (checks on
    consecutive sweeps alternate partial buffers) or, before a two-sweep
    launch, by a launch of its own.  The solve stops at the oracle's sweep."""
    import torch
    shape = (16, 12, 20)
    p = li.workload("C1", nx=20, ny=12, nz=16, dx=40.0, dy=30.0, dz=10.0, poisson_tol=1e-10,
                    poisson_scheme="chebyshev", poisson_check_every=every,
                    sweeps_per_launch=spl)
    rhs = li.random_field(shape, seed=24)
    phi_o, st_o = oracle_lib.poisson(p, rhs)
    sim = gpu.LES(p)
    phi_g, st_g, rc = sim.poisson_solve(torch.from_numpy(rhs))
    assert rc == 0 and st_o["status"] == 0 and st_g["status"] == 0
    assert st_g["sweeps"] == st_o["sweeps"]
    assert st_g["sweeps"] % every == 0
    assert rel(phi_g.cpu().numpy(), phi_o) <= 1e-11


def test_gated_guess_kept_rejected_and_capped(gpu, oracle_lib):
    """The guessed solve as the time step runs it (les_poisson_opts.use_guess
    = 2), FP64, against the oracle's: a guess that starts closer than the
    zero start is kept, one that starts farther is dropped, and a kept guess
    whose sweeps reach the cap is dropped and the sweeps repeated from the
    zero start, so the solve still ends converged.  The right-hand side is
    one eigenmode the fixed-weight sweep removes in a few sweeps; the guesses
    err by the slowest mode with horizontal and vertical structure."""
    import torch
    base = li.workload("C1", nx=16, ny=16, nz=16, dx=40.0, dy=40.0, dz=10.0,
                       poisson_scheme="jacobi", poisson_tol=1e-10, poisson_check_every=5)
    k, j, i = np.meshgrid(np.arange(16), np.arange(16), np.arange(16), indexing="ij")
    mode = (np.cos(2 * np.pi * 4 * i / 16) * np.cos(2 * np.pi * 4 * j / 16)
            * np.cos(np.pi * 8 * (k + 0.5) / 16))
    v = np.cos(2 * np.pi * (i + 0.5) / 16) * np.cos(np.pi * (k + 0.5) / 16)
    rhs = oracle_lib.laplacian(base, mode)
    phi0, s0 = oracle_lib.poisson(base, rhs)
    a = 0.5 * np.linalg.norm(rhs) / np.linalg.norm(oracle_lib.laplacian(base, v))
    budget = 2 * s0["sweeps"] + 1
    for cap, amp, bud, flag in ((100000, 1.0, 0, 1), (100000, 4.0, 0, 2), (100, 1.0, 0, 3),
                                (100000, 1.0, budget, 3)):
        p = dict(base, poisson_max_sweeps=cap)
        guess = phi0 + amp * a * v
        print(f"gated guess: cap {cap}, amplitude {amp}, budget {bud}", flush=True)
        phi_o, st_o = oracle_lib.poisson(p, rhs, guess=guess, gated=True, budget=bud)
        sim = gpu.LES(p)
        phi_g, st_g, rc = sim.poisson_solve(torch.from_numpy(rhs),
                                            torch.from_numpy(guess.copy()).cuda(), use_guess=2,
                                            budget=bud)
        assert st_o["guess"] == flag and st_g["guess"] == flag, (st_o, st_g)
        assert st_g["guess_sweeps"] == st_o["guess_sweeps"]
        assert st_g["status"] == 0 and rc == 0
        assert st_g["sweeps"] == st_o["sweeps"]
        assert rel(phi_g.cpu().numpy(), phi_o) <= 1e-11
        sim.close()


@pytest.mark.parametrize("scheme", ["jacobi", "chebyshev"])
def test_poisson_fp32_matches_oracle(gpu, oracle_lib, scheme):
    import torch
    shape = (16, 24, 40)
    p = li.workload("C1", nx=40, ny=24, nz=16, poisson_tol=1e-5, poisson_scheme=scheme,
                    precision="fp32")
    rhs = li.random_field(shape, seed=5)
    phi_o, st_o = oracle_lib.poisson(p, rhs)
    sim = gpu.LES(p)
    phi_g, st_g, rc = sim.poisson_solve(torch.from_numpy(rhs), fixed_sweeps=st_o["sweeps"])
    assert st_g["sweeps"] == st_o["sweeps"]
    e = rel(phi_g.double().cpu().numpy(), phi_o)
    assert e <= 1e-5, e
    assert st_g["res_norm"] <= 2e-5 * st_g["rhs_norm"]


def test_poisson_guess_and_zero_rhs(gpu, oracle_lib):
    import torch
    p = li.workload("C1", nx=16, ny=16, nz=16, poisson_tol=1e-10, poisson_scheme="chebyshev")
    rhs = li.random_field((16, 16, 16), seed=8)
    phi_o, _ = oracle_lib.poisson(p, rhs)
    sim = gpu.LES(p)
    guess = torch.from_numpy(phi_o.copy()).cuda()
    phi_g, st, _ = sim.poisson_solve(torch.from_numpy(rhs), guess, use_guess=True)
    assert st["sweeps"] == 0 and st["status"] == 0
    zero = torch.zeros((16, 16, 16), dtype=torch.float64)
    phi_z, st0, _ = sim.poisson_solve(zero, torch.full((16, 16, 16), 3.0, dtype=torch.float64,
                                                        device="cuda"), use_guess=True)
    assert st0["sweeps"] == 0 and torch.all(phi_z == 0)


def test_poisson_not_converged_and_nonfinite(gpu):
    import torch
    p = li.workload("C1", nx=8, ny=8, nz=8, poisson_max_sweeps=3, poisson_check_every=1)
    sim = gpu.LES(p)
    rhs = torch.from_numpy(li.random_field((8, 8, 8), seed=1))
    _, st, rc = sim.poisson_solve(rhs)
    assert rc == gpu.LES_WARN_NOT_CONVERGED and st["status"] == 1 and st["sweeps"] == 3
    bad = rhs.clone()
    bad[3, 3, 3] = float("nan")
    with pytest.raises(gpu.LesError) as ei:
        sim.poisson_solve(bad)
    assert ei.value.code == gpu.LES_ERR_NONFINITE


# ------------------------------------------------------- thermodynamics

@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_thermo_matches_oracle(gpu, oracle_lib, precision):
    import torch
    p = li.workload("C1m", precision=precision)
    st = li.initial_state(p)
    rng = np.random.default_rng(0)
    thl = st["thl"] + rng.uniform(-2, 2, st["thl"].shape)
    qt = np.clip(st["qt"] + rng.uniform(-3e-3, 3e-3, st["qt"].shape), 0, None)
    if precision == "fp32":
        # the oracle sees the same storage-rounded inputs as the kernel
        thl = thl.astype(np.float32).astype(np.float64)
        qt = qt.astype(np.float32).astype(np.float64)
    o = oracle_lib.thermo(p, thl, qt)
    sim = gpu.LES(p)
    g = sim.thermo(torch.from_numpy(thl), torch.from_numpy(qt))
    tol = 1e-12 if precision == "fp64" else 1e-6
    assert (o["ql"] > 0).mean() > 0.2
    for k in ("T", "ql", "b"):
        e = rel(g[k].double().cpu().numpy(), o[k])
        assert e <= tol, (k, e)
    if precision == "fp64":
        assert np.abs(g["T"].cpu().numpy() - o["T"]).max() <= 1e-9


def _heaviside_gap(oracle_lib, p, thl, qt):
    """Cells whose theta_l lies in the jump of theta_l*(T) at T_f under the
    Heaviside partition (all-ice just below T_f, all-liquid at it), widened
    by 1e-3 K: there the adjustment has no root (or one at the jump), and
    where the secant ends is not unique."""
    p0 = oracle_lib.reference_state(p)["p0"]
    tf = p["Tf"]
    gap = np.zeros(thl.shape, bool)
    for k, j, i in np.ndindex(*thl.shape):
        q, pk = qt[k, j, i], p0[k]
        liq = oracle_lib.theta_l(p, tf, max(0.0, q - oracle_lib.qv_sat(p, tf, pk)), 0.0, q, pk)
        ice = oracle_lib.theta_l(p, tf, 0.0, max(0.0, q - oracle_lib.qv_sat_ice(p, tf, pk)), q, pk)
        gap[k, j, i] = min(liq, ice) - 1e-3 < thl[k, j, i] < max(liq, ice) + 1e-3
    return gap, p0


@pytest.mark.parametrize("phase", ["heaviside", "ramp"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_thermo_ice_and_mixed_phase_matches_oracle(gpu, oracle_lib, phase, precision):
    """Cold states from all-ice through mixed phase to all-liquid (T about
    200 to 290 K over a 4 km column), saturated and not, in both partition
    modes (Sec. 2.2).  Under the Heaviside partition, cells inside the jump
    of theta_l* at T_f have no unique result: they are checked for validity
    (T within 1 K of T_f, liquid consistent with the side of T_f), the
    others element by element."""
    import torch
    p = li.workload("C1", nx=16, ny=16, nz=32, dz=125.0, theta0=265.0, phase=phase,
                    precision=precision)
    shape = (p["nz"], p["ny"], p["nx"])
    rng = np.random.default_rng(1)
    thl = rng.uniform(235.0, 290.0, shape)
    qt = rng.uniform(0.0, 10e-3, shape)
    if precision == "fp32":
        thl = thl.astype(np.float32).astype(np.float64)
        qt = qt.astype(np.float32).astype(np.float64)
    o = oracle_lib.thermo(p, thl, qt)
    assert (o["qi"] > 0).mean() > 0.3 and (o["ql"] > 0).mean() > 0.03
    if phase == "ramp":
        assert ((o["qi"] > 0) & (o["ql"] > 0)).mean() > 0.3
    sim = gpu.LES(p)
    g = {k: v.double().cpu().numpy() for k, v in sim.thermo(torch.from_numpy(thl),
                                                            torch.from_numpy(qt)).items()}
    keep = np.ones(shape, bool)
    if phase == "heaviside":
        gap, p0 = _heaviside_gap(oracle_lib, p, thl, qt)
        assert 0 < gap.sum() < 0.02 * gap.size
        keep = ~gap
        for k, j, i in zip(*np.nonzero(gap)):
            T = g["T"][k, j, i]
            assert abs(T - p["Tf"]) <= 1.0
            if T < p["Tf"]:
                assert g["ql"][k, j, i] == 0.0
            else:
                ql = max(0.0, qt[k, j, i] - oracle_lib.qv_sat(p, T, p0[k]))
                assert g["ql"][k, j, i] == pytest.approx(ql, rel=1e-5, abs=1e-12)
    tol = 1e-12 if precision == "fp64" else 1e-6
    for k in ("T", "ql", "b"):
        e = rel(g[k][keep], o[k][keep])
        assert e <= tol, (k, e)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-11), ("fp32", 1e-5)])
def test_step_cold_mixed_phase_matches_oracle(gpu, oracle_lib, precision, tol):
    """The cold workload: a cloud of liquid and ice partitioned by the ramp,
    with surface fluxes and radiation (liquid path), perturbed velocity."""
    p = li.workload("C1i", precision=precision, poisson_scheme="chebyshev",
                    poisson_tol=1e-9 if precision == "fp64" else 1e-6)
    if precision == "fp32":
        p = dict(p, nx=40, ny=24)
    st0 = with_velocity_noise(p, li.initial_state(p), 0.3, 14)
    if precision == "fp32":
        st0 = {k: v.astype(np.float32).astype(np.float64) for k, v in st0.items()}
    errs, *_, ost, gst = _compare_step(gpu, oracle_lib, p, st0, 2 if precision == "fp64" else 1,
                                       tol)
    if precision == "fp32":
        _fp32_bars(ost, gst)
    for k, e in errs.items():
        assert e <= tol, (k, e, errs)


# ------------------------------------------------------------ full step

def _compare_step(gpu, oracle_lib, p, st0, nsteps, tol, debug=False):
    ost = {k: v.copy() for k, v in st0.items()}
    recs, dbg = oracle_lib.step(p, ost, nsteps=nsteps, debug=debug)
    replay = [r["sweeps"] for r in recs]
    sim = gpu.LES(p, st0)
    rc, stats, grecs = sim.step(nsteps, replay=replay, records=True)
    gst = sim.state_numpy()
    errs = {k: rel(gst[k], ost[k]) for k in FIELDS}
    return errs, recs, grecs, sim, dbg, ost, gst


def test_step_c1_fp64_one_step(gpu, oracle_lib):
    p = li.workload("C1")
    st0 = li.initial_state(p)
    errs, recs, grecs, sim, dbg, ost, gst = _compare_step(gpu, oracle_lib, p, st0, 1, 1e-11, debug=True)
    g = sim.workspace_field("b_half").double().cpu().numpy()
    assert rel(g, dbg["b_half"]) <= 1e-11, rel(g, dbg["b_half"])
    # the sweeps' right-hand side: the centred rhs without its horizontal
    # mean per level (that part is solved exactly), relative to the whole
    g = sim.workspace_field("rhs").double().cpu().numpy()
    want = dbg["rhs"] - dbg["rhs"].mean(axis=(1, 2), keepdims=True)
    e = np.linalg.norm(g - want) / np.linalg.norm(dbg["rhs"])
    assert e <= 1e-11 and np.linalg.norm(want) > 1e-3 * np.linalg.norm(dbg["rhs"]), e
    for k, e in errs.items():
        assert e <= 1e-11, (k, e, errs)
    for a, b in zip(recs, grecs):
        assert a["sweeps"] == b["sweeps"]
        assert b["rhs_norm"] == pytest.approx(a["rhs_norm"], rel=1e-10)


@pytest.mark.parametrize("mean_mode", ["exact", "level", "swept"])
def test_step_c1m_fp64_all_physics(gpu, oracle_lib, mean_mode):
    """Saturated cells, surface fluxes, radiation, sponge, Coriolis, SGS with
    a perturbed velocity field; 2 steps, K = 2; the horizontally uniform
    part of each solve solved exactly or swept with the rest."""
    p = li.workload("C1m", poisson_tol=1e-9, poisson_scheme="chebyshev", mean_mode=mean_mode)
    st0 = with_velocity_noise(p, li.initial_state(p), 0.3, 4)
    errs, *_ = _compare_step(gpu, oracle_lib, p, st0, 2, 1e-11)
    for k, e in errs.items():
        assert e <= 1e-11, (k, e, errs)


@pytest.mark.parametrize("shape,advection,wall", [
    ((4, 5, 70), "quick", "no_slip"),     # every level within two cells of a wall
    ((7, 3, 130), "weno3", "free_slip"),  # a partial z chunk, three x segments, ragged
    ((9, 1, 66), "quick", "free_slip"),   # two-dimensional, a one-level z chunk
    ((6, 4, 64), "weno3", "no_slip"),     # whole x segments, two interior levels
])
def test_step_column_kernel_shapes_match_oracle(gpu, oracle_lib, shape, advection, wall):
    """The column-marching stencil kernels (advection, diffusion, SGS,
    divergence, projection) on launch shapes with ragged x segments, rows not
    a multiple of the block's four, partial z chunks and wall levels only:
    all moist physics, a perturbed velocity, two FP64 steps."""
    nz, ny, nx = shape
    p = li.workload("C1m", nx=nx, ny=ny, nz=nz, poisson_tol=1e-9, poisson_scheme="chebyshev",
                    advection=advection, wall=wall)
    st0 = with_velocity_noise(p, li.initial_state(p), 0.3, 31)
    errs, *_ = _compare_step(gpu, oracle_lib, p, st0, 2, 1e-11)
    for k, e in errs.items():
        assert e <= 1e-11, (k, e, errs)


@pytest.mark.parametrize("shape,dz", [
    ((300, 2, 5), 25.0),  # 16 waves of 19 levels: the levels past the 16 held in registers read again
    ((17, 3, 70), 50.0),  # two waves of 9 and 8 levels; a ragged second x segment
])
def test_step_radiation_columns_match_oracle(gpu, oracle_lib, shape, dz):
    """The radiative flux column (path sums per z chunk exchanged between the
    waves of a block, then each chunk marched from the path above it) on
    tall and short columns with a cloud layer: two FP64 steps."""
    nz, ny, nx = shape
    p = li.workload("C1m", nx=nx, ny=ny, nz=nz, dz=dz, poisson_tol=1e-9,
                    poisson_scheme="chebyshev")
    st0 = with_velocity_noise(p, li.initial_state(p), 0.3, 17)
    assert oracle_lib.thermo(p, st0["thl"], st0["qt"])["ql"].max() > 1e-4  # a cloud to absorb
    errs, *_ = _compare_step(gpu, oracle_lib, p, st0, 2, 1e-11)
    for k, e in errs.items():
        assert e <= 1e-11, (k, e, errs)


def test_step_c1_fp64_ten_steps(gpu, oracle_lib):
    """The configuration of the small parity case: 32^3, dt 0.5 s, tol 1e-8,
    fixed-weight Jacobi, 10 steps."""
    p = li.workload("C1")
    st0 = li.initial_state(p)
    errs, recs, grecs, *_ = _compare_step(gpu, oracle_lib, p, st0, 10, 1e-11)
    for k, e in errs.items():
        assert e <= 1e-11, (k, e, errs)
    assert all(r["status"] == 0 for r in grecs)


def test_step_fp32_matches_oracle(gpu, oracle_lib):
    """FP32 storage/stencils with FP64 reductions and saturation adjustment:
    per-field relative L2 error <= 1e-5 after one step (ragged 40x24x32 grid)."""
    p = li.workload("C1m", nx=40, ny=24, nz=32, precision="fp32", poisson_tol=1e-6,
                    poisson_scheme="chebyshev")
    st0 = with_velocity_noise(p, li.initial_state(p), 0.3, 7)
    *_, ost, gst = _compare_step(gpu, oracle_lib, p, st0, 1, 1e-5)
    _fp32_bars(ost, gst)


@pytest.mark.parametrize("guess", ["extrapolate", "previous"])
def test_step_guess_matches_oracle(gpu, oracle_lib, guess):
    """Initial guesses of the solves: the GPU forms the same starting
    iterate as the oracle (replayed sweep counts, FP64, 6 steps, all physics)."""
    p = li.workload("C1m", poisson_tol=1e-9, poisson_scheme="chebyshev", guess=guess)
    st0 = with_velocity_noise(p, li.initial_state(p), 0.3, 5)
    errs, recs, grecs, *_ = _compare_step(gpu, oracle_lib, p, st0, 6, 1e-11)
    for k, e in errs.items():
        assert e <= 1e-11, (k, e, errs)
    for a, b in zip(recs, grecs):
        assert b["res_norm"] == pytest.approx(a["res_norm"], rel=1e-6, abs=1e-12 * a["rhs_norm"])
        assert b["guess"] == a["guess"]


def test_step_guess_fp32_converges(gpu):
    """FP32, each solve of a guessed run stops at the tolerance, like the
    zero-guess run, and the two runs stay within tolerance-level distance."""
    base = li.workload("C1m", nx=40, ny=24, nz=32, precision="fp32", poisson_tol=1e-5,
                       poisson_scheme="chebyshev")
    out = {}
    for g in ("zero", "previous", "extrapolate"):
        p = dict(base, guess=g)
        sim = gpu.LES(p, li.initial_state(p))
        rc, stats, recs = sim.step(6, records=True)
        assert rc == gpu.LES_OK and stats["not_converged"] == 0
        for r in recs:
            assert r["res_norm"] <= p["poisson_tol"] * r["rhs_norm"]
        out[g] = sim.state_numpy()
    for g in ("previous", "extrapolate"):
        for k in FIELDS:
            assert rel_anom(out[g][k], out["zero"][k]) <= 1e-3, (g, k)


def test_step_weno3_fp64_matches_oracle(gpu, oracle_lib):
    """The paper's alternative advection (WENO3 faces, Lax-Friedrichs flux)
    for scalars and momentum: all physics, 2 steps, FP64 bar."""
    p = li.workload("C1m", poisson_tol=1e-9, poisson_scheme="chebyshev", advection="weno3")
    st0 = with_velocity_noise(p, li.initial_state(p), 0.3, 8)
    errs, *_ = _compare_step(gpu, oracle_lib, p, st0, 2, 1e-11)
    for k, e in errs.items():
        assert e <= 1e-11, (k, e, errs)


def test_step_weno3_fp32_matches_oracle(gpu, oracle_lib):
    p = li.workload("C1m", nx=40, ny=24, nz=32, precision="fp32", poisson_tol=1e-6,
                    poisson_scheme="chebyshev", advection="weno3")
    st0 = with_velocity_noise(p, li.initial_state(p), 0.3, 9)
    *_, ost, gst = _compare_step(gpu, oracle_lib, p, st0, 1, 1e-5)
    _fp32_bars(ost, gst)


# ------------------------------- validation cases (Sec. 3): uniform nu,
# free-slip walls, two-dimensional runs (ny = 1)

@pytest.mark.parametrize("case,advection", [("DC400", "quick"), ("RB400", "quick"),
                                            ("DC400", "weno3")])
def test_validation_case_fp64_matches_oracle(gpu, oracle_lib, case, advection):
    """Density current / rising bubble at 400 m (128 x 1 x 16, 50 x 1 x 25):
    four steps in FP64 against the oracle."""
    p = li.workload(case, precision="fp64", poisson_tol=1e-9, advection=advection)
    errs, recs, *_ = _compare_step(gpu, oracle_lib, p, li.initial_state(p), 4, 1e-11)
    assert all(r["sweeps"] > 0 for r in recs)
    for k, e in errs.items():
        assert e <= 1e-11, (k, e, errs)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-11), ("fp32", 1e-5)])
def test_free_slip_uniform_nu_3d_matches_oracle(gpu, oracle_lib, precision, tol):
    """Both options on a ragged three-dimensional grid with all moist physics
    and a perturbed velocity (every stress and advection term sees the wall
    parity of u and v)."""
    p = li.workload("C1m", nx=40, ny=24, nz=32, precision=precision,
                    poisson_tol=1e-9 if precision == "fp64" else 1e-6,
                    poisson_scheme="chebyshev", wall="free_slip", nu_const=3.0)
    st0 = with_velocity_noise(p, li.initial_state(p), 0.3, 12)
    if precision == "fp32":
        st0 = {k: v.astype(np.float32).astype(np.float64) for k, v in st0.items()}
    errs, *_, ost, gst = _compare_step(gpu, oracle_lib, p, st0, 2 if precision == "fp64" else 1,
                                       tol)
    if precision == "fp32":
        _fp32_bars(ost, gst)
    for k, e in errs.items():
        assert e <= tol, (k, e, errs)


def test_density_current_fp32_matches_oracle(gpu, oracle_lib):
    """The 200 m density current (256 x 1 x 32) in the FP32 path, two steps
    from the FP32-rounded initial state."""
    p = li.workload("DC200", precision="fp32")
    st0 = {k: v.astype(np.float32).astype(np.float64) for k, v in li.initial_state(p).items()}
    *_, ost, gst = _compare_step(gpu, oracle_lib, p, st0, 2, 1e-5)
    _fp32_bars(ost, gst)


def test_density_current_stays_mirror_symmetric_gpu(gpu):
    """200 steps (200 s) of the 200 m density current: theta_l and w
    symmetric and u antisymmetric about the domain centre to round-off."""
    p = li.workload("DC200", guess="previous")
    sim = gpu.LES(p, li.initial_state(p))
    rc, st, _ = sim.step(200, records=True)
    assert st["not_converged"] == 0
    st = sim.state_numpy()
    t, u, w = st["thl"][:, 0, :], st["u"][:, 0, :], st["w"][:, 0, :]
    assert np.abs(u).max() > 5.0
    dev = p["theta_bg"] - t
    assert np.abs(dev - dev[:, ::-1]).max() <= 1e-9 * np.abs(dev).max()
    assert np.abs(u + u[:, ::-1]).max() <= 1e-9 * np.abs(u).max()
    assert np.abs(w - w[:, ::-1]).max() <= 1e-9 * np.abs(w).max()


def test_two_dimensional_sweeps_one_vs_two_per_launch(gpu):
    """ny = 1 takes one-row sweep tiles; the fused two-sweep launch (its own
    tiles) gives the same iterates."""
    import torch
    out = []
    for spl in (1, 2):
        p = li.workload("DC200", sweeps_per_launch=spl)
        sim = gpu.LES(p)
        rhs = torch.from_numpy(li.random_field((p["nz"], p["ny"], p["nx"]), seed=5))
        phi, st, rc = sim.poisson_solve(rhs.float(), fixed_sweeps=60)
        out.append(phi.double().cpu().numpy())
    assert np.array_equal(out[0], out[1])


def test_poisson_streamed_wide_ragged_fp64(gpu, oracle_lib):
    """300 x 160 x 128 in FP64 (the four arrays exceed the Infinity Cache, so
    the streamed 256 x 4 tiles with a ragged last tile): 20 fixed sweeps
    against the oracle."""
    import torch
    shape = (128, 160, 300)
    p = li.workload("C1", nx=300, ny=160, nz=128, dx=35.0, dy=35.0, dz=5.0,
                    poisson_scheme="chebyshev")
    rhs = li.random_field(shape, seed=23)
    phi_o, _ = oracle_lib.poisson(p, rhs, fixed_sweeps=20)
    sim = gpu.LES(p)
    phi_g, st_g, rc = sim.poisson_solve(torch.from_numpy(rhs), fixed_sweeps=20)
    assert st_g["sweeps"] == 20
    e = rel(phi_g.cpu().numpy(), phi_o)
    assert e <= 1e-11, e


def test_all_options_fp32_matches_oracle(gpu, oracle_lib):
    """WENO3, the mixed-phase ramp, free-slip walls and a uniform viscosity
    together on the cold workload's physics, ragged grid, FP32."""
    p = li.workload("C1i", nx=40, ny=24, precision="fp32", poisson_scheme="chebyshev",
                    poisson_tol=1e-6, advection="weno3", wall="free_slip", nu_const=2.0)
    st0 = with_velocity_noise(p, li.initial_state(p), 0.3, 15)
    st0 = {k: v.astype(np.float32).astype(np.float64) for k, v in st0.items()}
    *_, ost, gst = _compare_step(gpu, oracle_lib, p, st0, 1, 1e-5)
    _fp32_bars(ost, gst)


def test_step_rest_state_steady(gpu):
    import torch
    p = li.workload("C1", nx=8, ny=8, nz=8, ug=0.0, vg=0.0, noise_thl=0.0, thl_ml=290.0,
                    dthl_inv=0.0, qt_ml=0.0, qt_ft=0.0, z_inv=1e9)
    st0 = li.initial_state(p)
    sim = gpu.LES(p, st0)
    rc, stats, recs = sim.step(3, records=True)
    gst = sim.state_numpy()
    for k in FIELDS:
        assert np.array_equal(gst[k], st0[k]), k
    assert all(r["sweeps"] == 0 for r in recs)


@pytest.mark.parametrize("scheme", ["quick", "weno3"])
def test_conservation_gpu(gpu, scheme):
    """Scalar domain integrals conserved without sources (FP64 path)."""
    p = li.workload("C1m", shf=0.0, lhf=0.0, rad_F0=0.0, poisson_tol=1e-6,
                    poisson_scheme="chebyshev", advection=scheme)
    st0 = with_velocity_noise(p, li.initial_state(p), 0.5, 2)
    sim = gpu.LES(p, st0)
    d0 = sim.diagnostics()
    sim.step(3)
    d1 = sim.diagnostics()
    assert abs(d1["mass_thl"] - d0["mass_thl"]) <= 1e-13 * abs(d0["mass_thl"])
    assert abs(d1["mass_qt"] - d0["mass_qt"]) <= 1e-13 * abs(d0["mass_qt"])


def test_diagnostics_match_oracle(gpu, oracle_lib):
    p = li.workload("C1m")
    st0 = with_velocity_noise(p, li.initial_state(p), 0.3, 3)
    o = oracle_lib.diagnostics(p, st0)
    sim = gpu.LES(p, st0)
    g = sim.diagnostics()
    for k in ("mass_thl", "mass_qt", "div_l2", "div_max", "cfl", "ke"):
        assert g[k] == pytest.approx(o[k], rel=1e-12), k
    for k, prof in o["profiles"].items():
        np.testing.assert_allclose(g["profiles"][k], prof, rtol=1e-11, atol=1e-15)


# ------------------------------------------- temporal blocking of sweeps

@pytest.mark.parametrize("precision,shape", [("fp64", (20, 36, 70)), ("fp32", (33, 20, 130)),
                                             ("fp32", (5, 6, 7))])
@pytest.mark.parametrize("scheme", ["jacobi", "chebyshev"])
def test_sweeps_per_launch_bitwise_equal(gpu, oracle_lib, precision, shape, scheme):
    """Fusing S sweeps in one launch changes only the launch shape: the
    iterates are bitwise equal for S = 1, 2, in fixed-count and in
    tolerance mode (ragged tiles in x, y and z)."""
    import torch
    nz, ny, nx = shape
    rhs = torch.from_numpy(li.random_field(shape, seed=13))
    ref = None
    for S in (1, 2):
        p = li.workload("C1", nx=nx, ny=ny, nz=nz, precision=precision, poisson_scheme=scheme,
                        poisson_tol=1e-5, sweeps_per_launch=S)
        sim = gpu.LES(p)
        phi_f, st_f, _ = sim.poisson_solve(rhs, fixed_sweeps=37)
        phi_t, st_t, _ = sim.poisson_solve(rhs)
        # the reported FP64 residual is that of the returned iterate: recompute
        # it from the (FP32-rounded or FP64) fixed-count iterate on the CPU
        if precision == "fp64":
            r = rhs.numpy() - rhs.numpy().mean() - oracle_lib.laplacian(p, phi_f.cpu().numpy())
            assert st_f["res_norm"] == pytest.approx(np.linalg.norm(r), rel=1e-10), S
        got = (phi_f.cpu().numpy(), phi_t.cpu().numpy(), st_t["sweeps"], st_t["res_norm"])
        if ref is None:
            ref = got
            assert st_f["sweeps"] == 37
            continue
        assert np.array_equal(got[0], ref[0]), S
        assert np.array_equal(got[1], ref[1]), S
        # same stopping sweep; the FP64 norm is summed over a launch-shape
        # dependent block decomposition, so only its last bits may differ
        assert got[2] == ref[2], S
        assert got[3] == pytest.approx(ref[3], rel=1e-12), S
