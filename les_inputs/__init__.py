"""Seeded synthetic inputs shared by the oracle and the HIP path.

This module holds workload parameters and the initial-state generator only.
It contains none of the method's arithmetic (no thermodynamics, no stencils,
no reference state): both the oracle and the library compute those on their
own from the parameters given here.

Workloads stand in for the stratocumulus case of the paper (Sec. 4, the
DYCOMS RF01 setup: a two-layer liquid-ice potential temperature / total water
profile, 289 K and 9 g/kg in the mixed layer).  The observational case
specification is not reproduced; the profile below is a synthetic stand-in.

Noise generator: splitmix64 (Steele, Lea & Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014), counter based:
    u = (splitmix64(seed ^ (field << 56) ^ idx) >> 11) * 2**-53,
    noise = a * (2u - 1).
"""
from __future__ import annotations

import copy

import numpy as np

# Field tags mixed into the counter so each field draws an independent stream.
FIELD_THL = 1
FIELD_QT = 2

_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)


def splitmix64(x: np.ndarray) -> np.ndarray:
    """splitmix64 finaliser applied elementwise to uint64 counters."""
    with np.errstate(over="ignore"):
        z = (np.asarray(x, dtype=np.uint64) + np.uint64(0x9E3779B97F4A7C15)) & _M64
        z = ((z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)) & _M64
        z = ((z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)) & _M64
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(seed: int, field: int, idx: np.ndarray) -> np.ndarray:
    """Uniform doubles in [0, 1) from the counter (seed, field, idx)."""
    key = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) ^ (np.uint64(field) << np.uint64(56))
    bits = splitmix64(key ^ np.asarray(idx, dtype=np.uint64))
    return (bits >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


# Thermodynamic constants and parameters (paper, Table 1).
TABLE1 = dict(
    p00=1.0e5,         # Pa
    theta0=290.0,      # K
    Rd=287.0,          # J/(kg K)
    Rv=461.89,
    cpd=1004.5,
    cpv=1859.5,
    cl=4181.0,
    ci=2100.0,
    Lv0=2.47e6,        # J/kg
    Ls0=2.83e6,
    Tf=273.15,         # K
    fcor=7.62e-5,      # 1/s
    g=9.81,            # m/s^2
    cs=0.18,
    Pr=0.4,
    Sc=0.4,
)

# Parameters every workload carries (values here are the defaults).
_BASE = dict(
    nx=32, ny=32, nz=32,
    dx=40.0, dy=40.0, dz=10.0, dt=0.5,
    n_subiter=2,
    poisson_scheme="jacobi",   # "jacobi" (fixed weight) or "chebyshev"
    poisson_tol=1e-8,
    poisson_max_sweeps=200000,
    poisson_check_every=25,
    jacobi_omega=0.0,          # 0 selects the closed-form optimum
    sweeps_per_launch=0,       # library launch shape only (0: its default)
    guess="zero",              # initial guess of the solves
    guess_passes=0,            # learned guess: network passes per solve (0 or 1: one)
    mean_mode="exact",         # parts of each solve solved exactly before the sweeps:
                               # "exact" (the horizontally uniform part, a 1D problem, and
                               # the vertically uniform part, a 2D one), "level" (the 1D
                               # part only) or "swept" (none)
    advection="quick",         # "quick" or "weno3" (WENO3 with Lax-Friedrichs flux)
    wall="no_slip",            # u, v at z = 0, H: "no_slip" or "free_slip"
    nu_const=0.0,              # > 0: uniform kinematic viscosity (m^2/s), no SGS model
    phase="heaviside",         # condensate partition: "heaviside" at T_f or "ramp"
    T_ice=233.15,              # ramp: all condensate is ice at and below T_ice (K)
    # forcing
    ug=7.0, vg=-5.0,
    shf=0.0, lhf=0.0,          # surface sensible / latent heat flux, W/m^2
    wsub_div=0.0,              # large-scale divergence D: w_sub = D z (downward)
    sponge_frac=0.05, sponge_max=0.25,
    rad_F0=0.0, rad_kappa=0.0,  # synthetic cloud-top longwave flux
    # saturation vapour pressure anchor (triple point) and secant stopping
    e_tr=611.657, T_tr=273.16,
    satadj_tol=1e-10, satadj_maxit=20,
    # initial state: "cloud_layer" (two-layer profile below) or "bubble"
    init="cloud_layer",
    # bubble: uniform theta_bg plus amp * cos^2(pi L / 2) for L <= 1,
    # L^2 = ((x - Lx/2) / xr)^2 + ((z - zc) / zr)^2, dry and at rest
    theta_bg=300.0, bubble_amp=0.0, bubble_xr=1.0, bubble_zr=1.0, bubble_zc=0.0,
    # two-layer profile
    z_inv=800.0, thl_ml=289.0, qt_ml=9.0e-3, dthl_inv=8.0, qt_ft=1.5e-3,
    noise_z=200.0, noise_thl=0.1, noise_qt=0.0,
    seed=1,
    precision="fp64",          # "fp64" or "fp32" (library only)
)
_BASE.update(TABLE1)

# Synthetic stand-ins for the paper's stratocumulus workloads.
WORKLOADS = {
    # 32^3, 40 m x 10 m, dt 0.5 s, tol 1e-8, fp64; Coriolis and sponge only.
    "C1": dict(),
    # Same grid with dz = 25 m (top at 800 m) so saturated cells exist.
    "C1m": dict(dz=25.0, noise_qt=2.5e-5, shf=15.0, lhf=115.0,
                rad_F0=60.0, rad_kappa=100.0),
    # 256x256x128, 35 m x 5 m, dt 0.3 s, tol 1e-6, fp32 storage.
    "C2": dict(nx=256, ny=256, nz=128, dx=35.0, dy=35.0, dz=5.0, dt=0.3,
               poisson_tol=1e-6, poisson_scheme="chebyshev", precision="fp32",
               poisson_max_sweeps=20000,
               noise_qt=2.5e-5, shf=15.0, lhf=115.0, rad_F0=60.0, rad_kappa=100.0,
               seed=2),
    # 512x512x256 precision study.
    "C3": dict(nx=512, ny=512, nz=256, dx=35.0, dy=35.0, dz=5.0, dt=0.3,
               poisson_tol=1e-6, poisson_scheme="chebyshev", precision="fp32",
               poisson_max_sweeps=40000,
               noise_qt=2.5e-5, shf=15.0, lhf=115.0, rad_F0=60.0, rad_kappa=100.0,
               seed=3),
    # 64^3 companion of C3 (same spacing and forcing) for oracle comparison.
    "C3s": dict(nx=64, ny=64, nz=64, dx=35.0, dy=35.0, dz=5.0, dt=0.3,
                poisson_tol=1e-6, poisson_scheme="chebyshev", precision="fp32",
                noise_qt=2.5e-5, shf=15.0, lhf=115.0, rad_F0=60.0, rad_kappa=100.0,
                seed=3),
    # Learned-guess evaluation grid (same as C2).
    "C4": dict(nx=256, ny=256, nz=128, dx=35.0, dy=35.0, dz=5.0, dt=0.3,
               poisson_tol=1e-6, poisson_scheme="chebyshev", precision="fp32",
               poisson_max_sweeps=20000,
               noise_qt=2.5e-5, shf=15.0, lhf=115.0, rad_F0=60.0, rad_kappa=100.0,
               seed=2000),
    # Cold mixed-phase variant of C1m (theta_l 258 K, 0.8 g/kg): a cloud of
    # liquid and ice from about 460 m to the top, partitioned by the ramp.
    "C1i": dict(dz=25.0, thl_ml=258.0, theta0=258.0, qt_ml=0.8e-3, noise_qt=2.5e-6,
                shf=15.0, lhf=115.0, rad_F0=60.0, rad_kappa=100.0, phase="ramp"),
    # The same cold profile on the 256x256x128 grid (thermodynamics timing).
    "C2i": dict(nx=256, ny=256, nz=128, dx=35.0, dy=35.0, dz=5.0, dt=0.3,
                poisson_tol=1e-6, poisson_scheme="chebyshev", precision="fp32",
                poisson_max_sweeps=20000, thl_ml=258.0, theta0=258.0, qt_ml=0.8e-3,
                z_inv=1e9, noise_qt=2.5e-6, shf=15.0, lhf=115.0, rad_F0=60.0,
                rad_kappa=100.0, phase="ramp", seed=2),
    # Largest single-GPU domain.
    "C5": dict(nx=1024, ny=1024, nz=256, dx=35.0, dy=35.0, dz=5.0, dt=0.3,
               poisson_tol=1e-6, poisson_scheme="chebyshev", precision="fp32",
               poisson_max_sweeps=80000,
               noise_qt=2.5e-5, shf=15.0, lhf=115.0, rad_F0=60.0, rad_kappa=100.0,
               seed=5),
}

# Dry validation cases (Sec. 3): two-dimensional (ny = 1) at uniform
# resolution h metres, the name carrying h.
#   DC<h>: density current, 51.2 km x 6.4 km, -15 K bubble of radii 4 km x
#          2 km centred 3 km up, uniform nu = 10 m^2/s, to t = 900 s.
#   RB<h>: rising bubble, 20 km x 10 km, +2 K bubble of radius 2 km centred
#          2 km up, uniform nu = 1 m^2/s, to t = 1000 s.
# Both: theta = 300 K background (also the reference state's theta0), no
# moisture, Coriolis, sponge, radiation or surface fluxes; free-slip walls;
# dt = h / 200 m/s (Courant number about 0.2 at the cases' peak speeds).
# FP64: their pressure correction is smooth on the grid scale, so FP32
# storage of it alone leaves a relative residual above the 1e-6 tolerance
# (5e-5 at 200 m, 1e-3 at 50 m for the density current).
DRY_CASES = {
    "DC": dict(Lx=51200.0, H=6400.0, bubble_amp=-15.0, bubble_xr=4000.0, bubble_zr=2000.0,
               bubble_zc=3000.0, nu_const=10.0, t_end=900.0),
    "RB": dict(Lx=20000.0, H=10000.0, bubble_amp=2.0, bubble_xr=2000.0, bubble_zr=2000.0,
               bubble_zc=2000.0, nu_const=1.0, t_end=1000.0),
}
DRY_RESOLUTIONS = (400, 200, 100, 50, 25, 10)


def _dry_workload(case: str, h: int) -> dict:
    d = DRY_CASES[case]
    return dict(nx=int(round(d["Lx"] / h)), ny=1, nz=int(round(d["H"] / h)),
                dx=float(h), dy=float(h), dz=float(h), dt=h / 200.0,
                poisson_scheme="chebyshev", poisson_tol=1e-6, poisson_max_sweeps=100000,
                precision="fp64", init="bubble", theta0=300.0, theta_bg=300.0,
                bubble_amp=d["bubble_amp"], bubble_xr=d["bubble_xr"],
                bubble_zr=d["bubble_zr"], bubble_zc=d["bubble_zc"],
                nu_const=d["nu_const"], wall="free_slip", ug=0.0, vg=0.0, fcor=0.0,
                sponge_max=0.0, noise_thl=0.0, noise_qt=0.0)


for _case in DRY_CASES:
    for _h in DRY_RESOLUTIONS:
        WORKLOADS[f"{_case}{_h}"] = _dry_workload(_case, _h)


def workload(name: str, **overrides) -> dict:
    """Full parameter dict of a named workload, with optional overrides."""
    if name not in WORKLOADS:
        raise KeyError(f"unknown workload {name!r}; known: {sorted(WORKLOADS)}")
    p = copy.deepcopy(_BASE)
    p.update(WORKLOADS[name])
    for k, v in overrides.items():
        if k not in p:
            raise KeyError(f"unknown parameter {k!r}")
        p[k] = v
    return p


def cell_heights(p: dict) -> np.ndarray:
    """Cell-centre heights z_k = (k + 1/2) dz (collocated grid)."""
    return (np.arange(p["nz"], dtype=np.float64) + 0.5) * p["dz"]


def initial_state(p: dict) -> dict:
    """Initial fields as float64 arrays of shape (nz, ny, nx), x fastest.

    init == "bubble": theta_l = theta_bg + bubble_amp cos^2(pi L / 2) where
    L <= 1 (L as in the parameters above, x measured from the domain centre
    Lx/2, which is a cell face when nx is even), q_t = 0, at rest.

    init == "cloud_layer": theta_l = thl_ml and q_t = qt_ml below z_inv; above it theta_l jumps by
    dthl_inv and then rises as (z - z_inv)^(1/3) K (z in m), q_t = qt_ft.
    Uniform noise of half-width noise_thl / noise_qt below noise_z.
    Velocity starts at the background wind (ug, vg, 0); p' starts at 0.
    """
    nx, ny, nz = p["nx"], p["ny"], p["nz"]
    shape = (nz, ny, nx)
    if p["init"] == "bubble":
        x = (np.arange(nx, dtype=np.float64) + 0.5) * p["dx"] - 0.5 * nx * p["dx"]
        zc = cell_heights(p) - p["bubble_zc"]
        L = np.sqrt((x[None, :] / p["bubble_xr"]) ** 2 + (zc[:, None] / p["bubble_zr"]) ** 2)
        pert = np.where(L <= 1.0, p["bubble_amp"] * np.cos(0.5 * np.pi * L) ** 2, 0.0)
        thl = p["theta_bg"] + np.broadcast_to(pert[:, None, :], shape)
        return dict(u=np.full(shape, p["ug"]), v=np.full(shape, p["vg"]), w=np.zeros(shape),
                    thl=np.ascontiguousarray(thl), qt=np.zeros(shape), p=np.zeros(shape))
    if p["init"] != "cloud_layer":
        raise ValueError(f"unknown init {p['init']!r}")
    z = cell_heights(p)[:, None, None] * np.ones((1, ny, nx))
    above = z >= p["z_inv"]
    thl = np.where(above, p["thl_ml"] + p["dthl_inv"]
                   + np.cbrt(np.maximum(z - p["z_inv"], 0.0)), p["thl_ml"])
    qt = np.where(above, p["qt_ft"], p["qt_ml"])
    # noise on the levels below noise_z only (the counter is the cell index,
    # so drawing it level by level gives the same values)
    nlow = int(np.count_nonzero(cell_heights(p) < p["noise_z"]))
    idx = np.arange(nx * ny * nlow, dtype=np.uint64).reshape(nlow, ny, nx)
    if p["noise_thl"] > 0 and nlow:
        r = uniform01(p["seed"], FIELD_THL, idx)
        thl[:nlow] = thl[:nlow] + p["noise_thl"] * (2.0 * r - 1.0)
    if p["noise_qt"] > 0 and nlow:
        r = uniform01(p["seed"], FIELD_QT, idx)
        qt[:nlow] = qt[:nlow] + p["noise_qt"] * (2.0 * r - 1.0)
    return dict(
        u=np.full(shape, p["ug"]),
        v=np.full(shape, p["vg"]),
        w=np.zeros(shape),
        thl=np.ascontiguousarray(thl),
        qt=np.ascontiguousarray(qt),
        p=np.zeros(shape),
    )


def random_field(shape, seed: int, field: int = 7, zero_mean: bool = True) -> np.ndarray:
    """Seeded uniform(-1, 1) field (e.g. a Poisson right-hand side)."""
    n = int(np.prod(shape))
    r = 2.0 * uniform01(seed, field, np.arange(n, dtype=np.uint64)) - 1.0
    r = r.reshape(shape)
    if zero_mean:
        r = r - r.mean()
    return r


FIELD_CNN = 11


def cnn_init(seed: int, blocks) -> np.ndarray:
    """Seeded initial parameters of a network, FP32 values as float64.

    blocks: sequence of (n_weights, fan_in, n_bias); weights are uniform in
    +-sqrt(3 / fan_in) (unit gain for a linear layer), biases zero.
    """
    out = []
    base = 0
    for nw, fan_in, nb in blocks:
        u = uniform01(seed, FIELD_CNN, np.arange(base, base + nw, dtype=np.uint64))
        base += nw
        out.append((2.0 * u - 1.0) * np.sqrt(3.0 / fan_in))
        out.append(np.zeros(nb))
    return np.concatenate(out).astype(np.float32).astype(np.float64)
