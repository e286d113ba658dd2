"""Pins of the FP64 CPU oracle against what the paper and mathematics fix.

Each test checks the oracle against something other than itself: closed
forms of the paper (Sec. 2.1 reference state, App. A stencil algebra),
textbook special cases, invariants (Sec. 2.4 conservation claim), brute
force (dense eigenvalues, bisection, FFT exact solves) and exact solutions of
ODEs discretised by the same time scheme.  CPU only.
"""
import math
import os

import numpy as np
import pytest

import les_inputs as li
from conftest import load_table1


def small(name="C1", **kw):
    return li.workload(name, **kw)


# ---------------------------------------------------------------- Table 1

def test_table1_matches_paper(oracle_lib):
    t1 = load_table1()
    p = li.workload("C1")
    for k, v in t1.items():
        assert p[k] == pytest.approx(v, rel=0, abs=0), k
    c = oracle_lib.make_cfg(p)
    for k, v in t1.items():
        assert getattr(c, k) == v


# ------------------------------------------------------ P1 reference state

def test_reference_state_closed_forms(oracle_lib):
    """T0 = theta0 - g z / cpd exactly follows from the two closed forms;
    rho0 = p0 / (Rd T0); dp0/dz = -rho0 g (hydrostatic balance)."""
    p = small(nz=64, dz=20.0)
    rs = oracle_lib.reference_state(p)
    z = li.cell_heights(p)
    np.testing.assert_allclose(rs["T0"], p["theta0"] - p["g"] * z / p["cpd"], rtol=1e-13)
    np.testing.assert_allclose(rs["rho0"] * rs["alpha0"], 1.0, rtol=1e-14)
    np.testing.assert_allclose(rs["rho0"], rs["p0"] / (p["Rd"] * rs["T0"]), rtol=1e-14)
    # p0 at the surface limit equals p00 (extrapolate two levels linearly)
    assert rs["p0"][0] < p["p00"]


def test_reference_state_hydrostatic_second_order(oracle_lib):
    errs = []
    for dz in (40.0, 20.0, 10.0):
        p = small(nz=int(1280 / dz), dz=dz)
        rs = oracle_lib.reference_state(p)
        dpdz = (rs["p0"][2:] - rs["p0"][:-2]) / (2 * dz)
        resid = dpdz + rs["rho0"][1:-1] * p["g"]
        errs.append(np.max(np.abs(resid)))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.6 < r1 < 4.4 and 3.6 < r2 < 4.4, errs


# ----------------------------------------------------- P2 thermodynamics

def test_theta_l_dry_is_textbook_theta(oracle_lib):
    p = small()
    for T, p0 in [(300.0, 1.0e5), (285.0, 9.0e4), (260.0, 7.5e4)]:
        th = oracle_lib.theta_l(p, T, 0.0, 0.0, 0.0, p0)
        assert th == pytest.approx(T * (p["p00"] / p0) ** (p["Rd"] / p["cpd"]), rel=1e-14)
        assert oracle_lib.exner(p, p0, 0.0, 0.0, 0.0) == pytest.approx(
            (p0 / p["p00"]) ** (287.0 / 1004.5), rel=1e-14)


def test_theta_l_liquid_lowers_theta(oracle_lib):
    """Condensate lowers theta_l by about L q_l / (c_p Pi) (Sec. 2.1)."""
    p = small()
    T, p0, qt, ql = 285.0, 9.5e4, 0.01, 1e-3
    th_dry = oracle_lib.theta_l(p, T, 0.0, 0.0, qt, p0)
    th_wet = oracle_lib.theta_l(p, T, ql, 0.0, qt, p0)
    approx = p["Lv0"] * ql / (p["cpd"] * (p0 / p["p00"]) ** 0.2857)
    assert th_dry - th_wet == pytest.approx(approx, rel=0.03)


def test_qv_sat_anchor_and_clausius_clapeyron(oracle_lib):
    p = small()
    eps = p["Rd"] / p["Rv"]

    def e_of(T, p0):
        q = oracle_lib.qv_sat(p, T, p0)
        return q * p0 / (eps + (1 - eps) * q)

    # triple-point anchor
    assert e_of(273.16, 1e5) == pytest.approx(611.657, rel=1e-12)
    # d ln e*/dT = L / (Rv T^2)
    for T in (275.0, 290.0, 300.0):
        h = 1e-3
        slope = (math.log(e_of(T + h, 1e5)) - math.log(e_of(T - h, 1e5))) / (2 * h)
        assert slope == pytest.approx(p["Lv0"] / (p["Rv"] * T * T), rel=1e-6)
    # magnitude: saturation vapour pressure at 20 C is about 2.34 kPa
    assert e_of(293.15, 1e5) == pytest.approx(2339.0, rel=0.02)


# ------------------------------------------------ P3 saturation adjustment

def test_satadj_round_trip_and_bisection(oracle_lib):
    p = small()
    rs_p = small(nz=130, dz=10.0)
    p0s = oracle_lib.reference_state(rs_p)["p0"]
    rng_T = np.linspace(270.0, 300.0, 13)
    rng_q = np.linspace(0.0, 0.02, 11)
    worst = 0.0
    nsat = 0
    for T in rng_T:
        for p0 in p0s[::13]:
            for qt in rng_q:
                qc = max(0.0, qt - oracle_lib.qv_star(p, T, p0))
                ql = qc if T >= p["Tf"] else 0.0
                qi = qc if T < p["Tf"] else 0.0
                thl = oracle_lib.theta_l(p, T, ql, qi, qt, p0)
                T2, ql2, qi2, it = oracle_lib.satadj(p, thl, qt, p0)
                worst = max(worst, abs(T2 - T))
                assert abs(ql2 - ql) <= 1e-11 and abs(qi2 - qi) <= 1e-11
                if qc > 0 and T >= p["Tf"]:
                    nsat += 1
                    assert 1 <= it <= 20
    assert nsat > 100
    assert worst <= 1e-9, worst


def test_satadj_matches_bisection(oracle_lib):
    """Independent root finder on theta_l*(T) - theta_l (Sec. 2.2)."""
    p = small()
    p0 = 9.3e4
    for thl, qt in [(289.0, 0.009), (289.0, 0.012), (292.0, 0.02), (289.0, 0.002)]:
        def f(T):
            qc = max(0.0, qt - oracle_lib.qv_sat(p, T, p0))
            return oracle_lib.theta_l(p, T, qc, 0.0, qt, p0) - thl
        lo, hi = 200.0, 350.0
        assert f(lo) < 0 < f(hi)
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            if f(mid) < 0:
                lo = mid
            else:
                hi = mid
        T, ql, qi, _ = oracle_lib.satadj(p, thl, qt, p0)
        assert T == pytest.approx(0.5 * (lo + hi), abs=1e-9)


# ------------------------------- ice and mixed phase (Sec. 2.2 partition)

def test_ice_saturation_clausius_clapeyron(oracle_lib):
    """Over ice the saturation vapour pressure follows Clausius-Clapeyron
    with the sublimation heat L_s0; it equals the liquid value at the triple
    point and lies below it at colder temperatures; at -20 C it is about
    103 Pa (published value 103.3 Pa, Murphy & Koop 2005)."""
    p = small()
    eps = p["Rd"] / p["Rv"]

    def e_of(T, p0):
        q = oracle_lib.qv_sat_ice(p, T, p0)
        return q * p0 / (eps + q * (1.0 - eps))

    for T in (230.0, 250.0, 265.0):
        h = 1e-3
        slope = (math.log(e_of(T + h, 1e5)) - math.log(e_of(T - h, 1e5))) / (2 * h)
        assert slope == pytest.approx(p["Ls0"] / (p["Rv"] * T * T), rel=1e-6)
        assert oracle_lib.qv_sat_ice(p, T, 8e4) < oracle_lib.qv_sat(p, T, 8e4)
    assert e_of(p["T_tr"], 1e5) == pytest.approx(p["e_tr"], rel=1e-14)
    assert oracle_lib.qv_sat_ice(p, p["T_tr"], 9e4) == pytest.approx(
        oracle_lib.qv_sat(p, p["T_tr"], 9e4), rel=1e-14)
    assert e_of(253.15, 1e5) == pytest.approx(103.3, rel=0.02)


def test_liquid_fraction_heaviside_and_ramp(oracle_lib):
    """Heaviside: liquid at and above T_f, ice below (Sec. 2.2).  Ramp: 1 at
    T_f, 0 at T_ice, linear between, clipped outside."""
    p = small()
    tf, ti = p["Tf"], p["T_ice"]
    assert oracle_lib.liquid_fraction(p, tf) == 1.0
    assert oracle_lib.liquid_fraction(p, tf - 1e-9) == 0.0
    r = small(phase="ramp")
    assert oracle_lib.liquid_fraction(r, tf) == 1.0
    assert oracle_lib.liquid_fraction(r, tf + 5) == 1.0
    assert oracle_lib.liquid_fraction(r, ti) == 0.0
    assert oracle_lib.liquid_fraction(r, ti - 5) == 0.0
    for f in (0.1, 0.5, 0.8):
        assert oracle_lib.liquid_fraction(r, ti + f * (tf - ti)) == pytest.approx(f, abs=1e-14)
    # the saturation humidity blends the two phases with the same weight
    T, p0 = ti + 0.25 * (tf - ti), 8.5e4
    assert oracle_lib.qv_star(r, T, p0) == pytest.approx(
        0.25 * oracle_lib.qv_sat(r, T, p0) + 0.75 * oracle_lib.qv_sat_ice(r, T, p0), rel=1e-14)


def test_mixed_phase_round_trip_and_bisection(oracle_lib):
    """Ramp partition: theta_l*(T) is continuous through the mixed-phase
    range, so theta_l built from (T, q_t) at saturation gives back T, and
    the secant root equals an independent bisection root.  Condensate splits
    as lambda(T) : 1 - lambda(T) and q_v + q_l + q_i = q_t."""
    p = small(phase="ramp")
    p0s = oracle_lib.reference_state(small(nz=130, dz=10.0, phase="ramp"))["p0"][::26]
    worst = 0.0
    nmix = 0
    for T in np.linspace(215.0, 290.0, 16):
        lam = oracle_lib.liquid_fraction(p, T)
        for p0 in p0s:
            qs = oracle_lib.qv_star(p, T, p0)
            for qt in (0.5 * qs, 1.5 * qs, 3.0 * qs):
                qc = max(0.0, qt - qs)
                thl = oracle_lib.theta_l(p, T, lam * qc, (1 - lam) * qc, qt, p0)
                T2, ql2, qi2, it = oracle_lib.satadj(p, thl, qt, p0)
                worst = max(worst, abs(T2 - T))
                assert ql2 == pytest.approx(lam * qc, abs=1e-12)
                assert qi2 == pytest.approx((1 - lam) * qc, abs=1e-12)
                if qc > 0 and 0 < lam < 1:
                    nmix += 1
                    assert ql2 > 0 and qi2 > 0
                    qv = oracle_lib.qv_star(p, T2, p0)
                    assert qv + ql2 + qi2 == pytest.approx(qt, rel=1e-9)

                def f(Tx):
                    lx = oracle_lib.liquid_fraction(p, Tx)
                    qx = max(0.0, qt - oracle_lib.qv_star(p, Tx, p0))
                    return oracle_lib.theta_l(p, Tx, lx * qx, (1 - lx) * qx, qt, p0) - thl
                lo, hi = 150.0, 350.0
                assert f(lo) < 0 < f(hi)
                for _ in range(200):
                    mid = 0.5 * (lo + hi)
                    lo, hi = (mid, hi) if f(mid) < 0 else (lo, mid)
                assert T2 == pytest.approx(0.5 * (lo + hi), abs=1e-9)
    assert nmix >= 20
    assert worst <= 1e-9, worst


def test_cold_cloud_layer_is_mixed_phase(oracle_lib):
    """The cold workload (theta_l 258 K, 0.8 g/kg): temperatures inside the
    ramp, a cloud of liquid and ice in the upper part, the ice share growing
    with height as the air cools."""
    p = small("C1i")
    st = li.initial_state(p)
    th = oracle_lib.thermo(p, st["thl"], st["qt"])
    assert p["T_ice"] < th["T"].min() and th["T"].max() < p["Tf"]
    ql, qi = th["ql"].mean(axis=(1, 2)), th["qi"].mean(axis=(1, 2))
    cloudy = np.where(ql + qi > 0)[0]
    assert 300.0 < li.cell_heights(p)[cloudy.min()] < 600.0
    share = qi[cloudy] / (ql[cloudy] + qi[cloudy])
    assert np.all(share > 0.3) and np.all(share < 0.7) and np.all(np.diff(share) > 0)


def test_cloud_layer_exists_in_stratocumulus_profile(oracle_lib):
    """The mixed layer (289 K, 9 g/kg) saturates well below the inversion."""
    p = small("C1m")
    st = li.initial_state(p)
    th = oracle_lib.thermo(p, st["thl"], st["qt"])
    qlm = th["ql"].mean(axis=(1, 2))
    z = li.cell_heights(p)
    cloudy = z[qlm > 0]
    assert cloudy.size > 0
    assert 350.0 < cloudy.min() < 600.0 and cloudy.max() < 800.0
    assert 4e-4 < qlm.max() < 1.2e-3
    assert np.all(th["qi"] == 0.0)


def test_buoyancy_zero_at_reference(oracle_lib):
    p = small()
    shape = (p["nz"], p["ny"], p["nx"])
    th = oracle_lib.thermo(p, np.full(shape, p["theta0"]), np.zeros(shape))
    assert np.all(th["b"] == 0.0)
    rs = oracle_lib.reference_state(p)
    np.testing.assert_allclose(th["T"][:, 0, 0], rs["T0"], rtol=1e-15)


def _check_buoyancy_dry(lib):
    """Dry air (q_t = 0) at the reference pressure: alpha / alpha0 = T / T0
    = theta / theta0, so b = g (theta_l - theta0) / theta0 exactly, the
    textbook dry buoyancy (Sec. 2.1 buoyancy and equation of state)."""
    p = small(nx=4, ny=3, nz=32)
    shape = (p["nz"], p["ny"], p["nx"])
    rng = np.random.default_rng(21)
    dth = rng.uniform(0.5, 3.0, shape) * rng.choice([-1.0, 1.0], shape)
    th = lib.thermo(p, p["theta0"] + dth, np.zeros(shape))
    np.testing.assert_allclose(th["b"], p["g"] * dth / p["theta0"], rtol=1e-10, atol=0)


def _moist_states(p):
    """Unsaturated moist cells (2-6 g/kg) in the lower half of the column and
    cloudy cells (10-14 g/kg) in the upper half, theta_l within 2 K of theta0."""
    shape = (p["nz"], p["ny"], p["nx"])
    rng = np.random.default_rng(22)
    upper = (np.arange(p["nz"]) >= p["nz"] // 2)[:, None, None]
    qt = np.where(upper, rng.uniform(10e-3, 14e-3, shape), rng.uniform(2e-3, 6e-3, shape))
    thl = p["theta0"] + rng.uniform(-2.0, 2.0, shape)
    return thl, qt


def _check_buoyancy_moist(lib):
    """Moist air: the textbook buoyancy with water-vapour and condensate
    loading, linearised in small perturbations,
        b ~ g [ (T - T0)/T0 + (R_v/R_d - 1) q_v - q_c ],
    holds up to its second-order remainder g |(T - T0)/T0| |(R_v/R_d - 1) q_v - q_c|.
    T and q_c come from the saturation adjustment (pinned by the round trip
    and bisection tests), T0 from the closed form T0 = theta0 - g z / c_pd.
    A condensate left out of R_m shifts b by g q_c R_v/R_d (~0.02 m/s^2 per
    g/kg), a reference temperature in place of T by g (T - T0)/T0; both are
    first order and exceed the remainder many times over."""
    p = small(nx=4, ny=4, nz=32, dz=25.0)
    thl, qt = _moist_states(p)
    th = lib.thermo(p, thl, qt)
    qc = th["ql"] + th["qi"]
    cloudy = qc > 5e-4
    assert cloudy.mean() > 0.3 and ((qc == 0) & (qt > 2e-3)).mean() > 0.3
    T0 = (p["theta0"] - p["g"] * li.cell_heights(p) / p["cpd"])[:, None, None]
    dT = th["T"] / T0 - 1.0
    a = (p["Rv"] / p["Rd"] - 1.0) * (qt - qc) - qc
    lin = p["g"] * (dT + a)
    bound = p["g"] * np.abs(dT) * np.abs(a) * (1 + 1e-9) + 1e-13
    assert np.all(np.abs(th["b"] - lin) <= bound), np.max(np.abs(th["b"] - lin) / bound)
    assert np.max(bound) < 2e-3


def _check_radiation_heating(lib):
    """One step with K = 1 of a column at rest with no advection, diffusion,
    surface flux or subsidence changes theta_l only by the radiative source
    of the Sec. 2.1 theta_l equation: rho0 d theta_l / dt =
    -(c_pm Pi)^-1 d F / dz, F the synthetic longwave flux at the faces.
    c_pm Pi is taken from the theta_l definition solved for Pi,
    c_pm Pi = (c_pm T - L_v0 q_l) / theta_l, not from the Exner power, so a
    heating that uses c_pm alone (Pi dropped, 2-5 % off here) fails."""
    p = small("C1m", nx=2, ny=2, n_subiter=1, ug=0.0, vg=0.0, fcor=0.0, shf=0.0, lhf=0.0,
              noise_thl=0.0, noise_qt=0.0, cs=0.0, sponge_max=0.0, poisson_tol=1e-8,
              poisson_scheme="chebyshev")
    st = li.initial_state(p)
    thl0, qt = st["thl"][:, 0, 0].copy(), st["qt"][:, 0, 0].copy()
    th = lib.thermo(p, st["thl"], st["qt"])
    lib.step(p, st, nsteps=1)
    rs = lib.reference_state(p)
    T, ql = th["T"][:, 0, 0], th["ql"][:, 0, 0]
    assert ql.max() > 3e-4 and np.all(th["qi"] == 0)
    cpm = (1 - qt) * p["cpd"] + (qt - ql) * p["cpv"] + ql * p["cl"]
    cpm_pi = (cpm * T - p["Lv0"] * ql) / thl0
    nz = p["nz"]
    F = np.empty(nz + 1)
    F[nz] = p["rad_F0"]
    path = 0.0
    for k in range(nz - 1, -1, -1):
        path += rs["rho0"][k] * ql[k] * p["dz"]
        F[k] = p["rad_F0"] * np.exp(-p["rad_kappa"] * path)
    expect = -p["dt"] / rs["rho0"] * (F[1:] - F[:-1]) / (p["dz"] * cpm_pi)
    got = st["thl"][:, 0, 0] - thl0
    assert np.abs(expect).max() > 1e-4
    np.testing.assert_allclose(got, expect, rtol=1e-7, atol=1e-12)
    assert np.all(st["thl"] == st["thl"][:, :1, :1])


def test_buoyancy_dry_is_textbook(oracle_lib):
    _check_buoyancy_dry(oracle_lib)


def test_buoyancy_moist_linearisation(oracle_lib):
    _check_buoyancy_moist(oracle_lib)


def test_radiation_heating_per_level(oracle_lib):
    _check_radiation_heating(oracle_lib)


# Planted mistakes: a copy of the oracle with one plausible error each,
# built on the CPU, must fail the pins above.
PLANTED = {
    "condensate_left_out_of_Rm": (
        "double Rm = (1.0 - qt[n]) * c->Rd + (qt[n] - qlc - qic) * c->Rv;",
        "double Rm = (1.0 - qt[n]) * c->Rd + qt[n] * c->Rv;",
        [_check_buoyancy_moist]),
    "reference_temperature_in_alpha": (
        "double alpha = Rm * Tc / P.p0[k];",
        "double alpha = Rm * P.T0[k] / P.p0[k];",
        [_check_buoyancy_dry, _check_buoyancy_moist]),
    "exner_dropped_from_radiative_heating": (
        "return cpm * oracle_exner(c, p0, qt, ql, qi);",
        "return cpm;",
        [_check_radiation_heating]),
}


def _build_planted(tmp_path, old, new):
    import shutil
    import subprocess
    from oracle import build as obuild
    src = os.path.join(os.path.dirname(obuild.HERE), "oracle")
    for f in os.listdir(src):
        if f.endswith((".c", ".h")):
            shutil.copy(os.path.join(src, f), tmp_path / f)
    path = tmp_path / "les_oracle.c"
    text = path.read_text()
    assert text.count(old) == 1, old
    path.write_text(text.replace(old, new))
    lib = str(tmp_path / "liboracle_planted.so")
    subprocess.run(obuild.CMD + [lib, str(path), str(tmp_path / "cnn_oracle.c"), "-lm"],
                   check=True)
    return lib


@pytest.mark.parametrize("name", sorted(PLANTED))
def test_planted_thermodynamics_mistakes_fail_pins(oracle_lib, tmp_path, name):
    old, new, checks = PLANTED[name]
    lib = _build_planted(tmp_path, old, new)
    with oracle_lib.variant(lib):
        for check in checks:
            with pytest.raises(AssertionError):
                check(oracle_lib)


# ---------------------------------------------------- discrete operators

def _modes(p, ax, m):
    """Eigenfunction along one axis: periodic cos(2 pi m l / N) or, on the
    mirror axis z, cos(pi m (l + 1/2) / N); returns (field, theta)."""
    nx, ny, nz = p["nx"], p["ny"], p["nz"]
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    if ax == 0:
        th = 2 * np.pi * m / nx
        return np.cos(th * i), th
    if ax == 1:
        th = 2 * np.pi * m / ny
        return np.cos(th * j), th
    th = np.pi * m / nz
    return np.cos(th * (k + 0.5)), th


@pytest.mark.parametrize("ax", [0, 1, 2])
def test_app_a_symbol(oracle_lib, ax):
    """App. A: C = wide - compact has symbol (1 - cos theta)^2 / Delta^2;
    the checkerboard gives 4 / Delta^2."""
    p = small(nx=8, ny=12, nz=10, dx=40.0, dy=30.0, dz=10.0)
    d = (p["dx"], p["dy"], p["dz"])[ax]
    n = (p["nx"], p["ny"], p["nz"])[ax]
    for m in range(0, n if ax == 2 else n // 2 + 1):
        f, th = _modes(p, ax, m)
        out = oracle_lib.app_a(p, f)
        np.testing.assert_allclose(out, (1 - np.cos(th)) ** 2 / d ** 2 * f, atol=1e-14 / d ** 2)
        lap = oracle_lib.laplacian(p, f)
        np.testing.assert_allclose(lap, -(2 - 2 * np.cos(th)) / d ** 2 * f, atol=1e-14 / d ** 2)
    if ax < 2:
        f, th = _modes(p, ax, n // 2)
        assert th == pytest.approx(np.pi)
        np.testing.assert_allclose(oracle_lib.app_a(p, f), 4.0 / d ** 2 * f, atol=1e-14)


def test_divergence_of_gradient_is_wide_laplacian(oracle_lib):
    """div_c grad_c = compact Laplacian + C on periodic axes (App. A)."""
    p = small(nx=8, ny=8, nz=8)
    rng = np.random.default_rng(0)
    f = rng.standard_normal((8, 8, 8))
    f = np.repeat(f[:1], 8, axis=0)  # z-uniform: only periodic axes matter
    gx = (np.roll(f, -1, 2) - np.roll(f, 1, 2)) / (2 * p["dx"])
    gy = (np.roll(f, -1, 1) - np.roll(f, 1, 1)) / (2 * p["dy"])
    wide = oracle_lib.divergence(p, gx, gy, np.zeros_like(f))
    np.testing.assert_allclose(wide, oracle_lib.laplacian(p, f) + oracle_lib.app_a(p, f),
                               atol=1e-16)


def test_jacobi_bounds_brute_force(oracle_lib):
    """Closed-form extreme eigenvalues of -D^{-1} L equal those of the dense
    matrix assembled column by column from the oracle's Laplacian."""
    for (nx, ny, nz) in [(4, 5, 4), (6, 4, 5)]:
        p = small(nx=nx, ny=ny, nz=nz, dx=40.0, dy=35.0, dz=10.0)
        n = nx * ny * nz
        A = np.zeros((n, n))
        for q in range(n):
            e = np.zeros(n)
            e[q] = 1.0
            A[:, q] = oracle_lib.laplacian(p, e.reshape(nz, ny, nx)).ravel()
        d = 2 / p["dx"] ** 2 + 2 / p["dy"] ** 2 + 2 / p["dz"] ** 2
        ev = np.sort(np.linalg.eigvalsh(-A / d))
        assert abs(ev[0]) < 1e-12 and ev[1] > 1e-6
        lo, hi = oracle_lib.jacobi_bounds(dict(p, mean_mode="level"))
        assert lo == pytest.approx(ev[1], rel=1e-10)
        assert hi == pytest.approx(ev[-1], rel=1e-10)
        # With both uniform parts solved exactly the sweeps act on the fields
        # with zero horizontal mean on every level and zero vertical mean in
        # every column: the operator restricted there (an orthonormal basis
        # of that subspace, from the projector's eigenvectors) has the
        # smallest eigenvalue the closed form gives.
        k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
        k, j, i = k.ravel(), j.ravel(), i.ravel()
        col = j * nx + i
        Pm = (np.eye(n) - (k[:, None] == k[None, :]) / (nx * ny)
              - (col[:, None] == col[None, :]) / nz + 1.0 / n)
        w, Q = np.linalg.eigh(Pm)
        B = Q[:, w > 0.5]
        evs = np.sort(np.linalg.eigvalsh(B.T @ (-A / d) @ B))
        lo2, hi2 = oracle_lib.jacobi_bounds(dict(p, mean_mode="exact"))
        assert lo2 == pytest.approx(evs[0], rel=1e-10)
        assert hi2 == pytest.approx(evs[-1], rel=1e-10)
        assert lo2 > 2 * lo


def test_vertical_mode_solve_matches_fft(oracle_lib):
    """The vertically uniform part's exact solution (real Fourier basis)
    against numpy's complex FFT solution of the 2D periodic problem, on
    even and odd sizes and a one-row (x-z) grid."""
    for (ny, nx) in [(8, 8), (6, 10), (7, 5), (1, 12)]:
        p = small(nx=nx, ny=ny, nz=4, dx=40.0, dy=30.0)
        rv = li.random_field((1, ny, nx), seed=17)[0]
        pv = oracle_lib.vertical_mode_solve(p, rv)
        F = np.fft.fft2(rv)
        ky = 2 * np.pi * np.fft.fftfreq(ny)
        kx = 2 * np.pi * np.fft.fftfreq(nx)
        lam = -((2 - 2 * np.cos(ky))[:, None] / p["dy"] ** 2
                + (2 - 2 * np.cos(kx))[None, :] / p["dx"] ** 2)
        lam[0, 0] = 1.0
        F = F / lam
        F[0, 0] = 0.0
        exact = np.real(np.fft.ifft2(F))
        np.testing.assert_allclose(pv, exact, rtol=0, atol=1e-12 * np.abs(exact).max())


def test_vertically_uniform_rhs_needs_no_sweep(oracle_lib):
    """A right-hand side constant in z is the vertically uniform part only:
    with both uniform parts exact it is solved with no sweep, every level
    equal to the 2D solution."""
    nz, ny, nx = 6, 10, 12
    p = small(nx=nx, ny=ny, nz=nz, poisson_tol=1e-12, mean_mode="exact")
    r2 = li.random_field((1, ny, nx), seed=19)
    rhs = np.repeat(r2, nz, axis=0)
    phi, st = oracle_lib.poisson(p, rhs)
    assert st["status"] == 0 and st["sweeps"] == 0
    pv = oracle_lib.vertical_mode_solve(p, r2[0])
    np.testing.assert_allclose(phi, np.broadcast_to(pv, phi.shape), rtol=0,
                               atol=1e-12 * np.abs(pv).max())


def test_exact_uniform_parts_cut_the_sweeps(oracle_lib):
    """On the benchmark's spacing (35 m x 35 m x 5 m), with the horizontal
    scales far larger than the vertical ones, the slowest modes are the
    vertically uniform ones; solving them exactly raises the smallest
    eigenvalue the sweeps see from lambda_h(1) to lambda_h(1) + lambda_z(1)
    and the sweeps to the same tolerance fall about sqrt of that ratio."""
    shape = (32, 64, 64)
    base = dict(nx=64, ny=64, nz=32, precision="fp64", poisson_tol=1e-8)
    rhs = li.random_field(shape, seed=3)
    out = {}
    for mm in ("level", "exact"):
        p = li.workload("C2", mean_mode=mm, **base)
        phi, st = oracle_lib.poisson(p, rhs)
        assert st["status"] == 0
        out[mm] = (phi, st["sweeps"], oracle_lib.jacobi_bounds(p)[0])
    ratio = out["exact"][2] / out["level"][2]
    assert ratio > 40
    assert out["exact"][1] * 5 < out["level"][1]
    np.testing.assert_allclose(out["exact"][0], out["level"][0], rtol=0,
                               atol=1e-6 * np.abs(out["level"][0]).max())


# ------------------------------------------------------ P7 Poisson exact

def fft_poisson(p, rhs):
    """Exact solution of the compact Laplacian with periodic x, y and
    mirror-Neumann z: extend z symmetrically to 2 nz (half-sample), solve
    mode by mode with eigenvalues -sum (2 - 2 cos theta) / Delta^2."""
    nz = rhs.shape[0]
    ext = np.concatenate([rhs, rhs[::-1]], axis=0)
    F = np.fft.fftn(ext)
    kz = 2 * np.pi * np.fft.fftfreq(2 * nz)
    ky = 2 * np.pi * np.fft.fftfreq(rhs.shape[1])
    kx = 2 * np.pi * np.fft.fftfreq(rhs.shape[2])
    lam = -((2 - 2 * np.cos(kz))[:, None, None] / p["dz"] ** 2
            + (2 - 2 * np.cos(ky))[None, :, None] / p["dy"] ** 2
            + (2 - 2 * np.cos(kx))[None, None, :] / p["dx"] ** 2)
    lam[0, 0, 0] = 1.0
    F = F / lam
    F[0, 0, 0] = 0.0
    return np.real(np.fft.ifftn(F))[:nz]


@pytest.mark.parametrize("shape", [(8, 8, 8), (10, 12, 16)])
@pytest.mark.parametrize("scheme", ["jacobi", "chebyshev"])
@pytest.mark.parametrize("mean_mode", ["exact", "level", "swept"])
def test_poisson_matches_fft(oracle_lib, shape, scheme, mean_mode):
    nz, ny, nx = shape
    p = small(nx=nx, ny=ny, nz=nz, dx=40.0, dy=30.0, dz=10.0, poisson_tol=1e-12,
              poisson_scheme=scheme, mean_mode=mean_mode)
    rhs = li.random_field(shape, seed=11)
    exact = fft_poisson(p, rhs)
    phi, st = oracle_lib.poisson(p, rhs)
    assert st["status"] == 0
    assert st["res_norm"] <= 1e-12 * st["rhs_norm"]
    np.testing.assert_allclose(phi, exact, atol=1e-10 * np.abs(exact).max())
    assert abs(phi.mean()) < 1e-15 * np.abs(exact).max() * 10


def test_poisson_fully_periodic_limit(oracle_lib):
    """A z-uniform right-hand side reduces the problem to the 2D periodic one."""
    p = small(nx=8, ny=8, nz=4, poisson_tol=1e-12)
    r2 = li.random_field((1, 8, 8), seed=5)
    rhs = np.repeat(r2, 4, axis=0)
    phi, st = oracle_lib.poisson(p, rhs)
    F = np.fft.fft2(r2[0])
    ky = 2 * np.pi * np.fft.fftfreq(8)
    lam = -((2 - 2 * np.cos(ky))[:, None] / p["dy"] ** 2 + (2 - 2 * np.cos(ky))[None, :] / p["dx"] ** 2)
    lam[0, 0] = 1
    F = F / lam
    F[0, 0] = 0
    exact = np.real(np.fft.ifft2(F))
    for k in range(4):
        np.testing.assert_allclose(phi[k], exact, atol=1e-10 * np.abs(exact).max())


def test_mean_mode_of_a_horizontally_uniform_rhs(oracle_lib):
    """A right-hand side of z alone is the horizontally uniform mode only:
    the exact start of that mode solves it with no sweep, and it equals the
    dense minimum-norm (zero-mean) solution of the one-dimensional mirror-
    Neumann second difference.  Sweeping that mode instead takes hundreds of
    sweeps."""
    nz, ny, nx = 24, 5, 6
    p = small(nx=nx, ny=ny, nz=nz, dz=7.0, poisson_tol=1e-12, mean_mode="exact")
    rng = np.random.default_rng(8)
    r = rng.standard_normal(nz)
    r -= r.mean()
    rhs = np.broadcast_to(r[:, None, None], (nz, ny, nx)).copy()
    phi, st = oracle_lib.poisson(p, rhs)
    assert st["status"] == 0 and st["sweeps"] == 0
    A = (np.diag(-2.0 * np.ones(nz)) + np.diag(np.ones(nz - 1), 1) + np.diag(np.ones(nz - 1), -1))
    A[0, 0] = A[-1, -1] = -1.0
    exact = np.linalg.pinv(A / p["dz"] ** 2) @ r
    np.testing.assert_allclose(phi, np.broadcast_to(exact[:, None, None], rhs.shape),
                               rtol=0, atol=1e-11 * np.abs(exact).max())
    _, st2 = oracle_lib.poisson(small(nx=nx, ny=ny, nz=nz, dz=7.0, poisson_tol=1e-12,
                                      mean_mode="swept"), rhs)
    assert st2["status"] == 0 and st2["sweeps"] > 100


def test_mean_mode_ignores_level_means_of_a_guess(oracle_lib):
    """With both uniform parts solved exactly, a guess's horizontal means per
    level and vertical means per column play no part: adding any profile of
    z and any field of (x, y) to it changes neither the sweeps nor the
    solution."""
    shape = (12, 10, 14)
    p = small(nx=14, ny=10, nz=12, poisson_tol=1e-10, poisson_scheme="chebyshev",
              mean_mode="exact")
    rhs = li.random_field(shape, seed=12)
    g = li.random_field(shape, seed=13) * 40.0
    prof = np.linspace(-300.0, 500.0, 12)[:, None, None]
    plane = 200.0 * li.random_field((1, 10, 14), seed=14)
    a, sa = oracle_lib.poisson(p, rhs, guess=g)
    b, sb = oracle_lib.poisson(p, rhs, guess=g + prof + plane)
    assert sa["sweeps"] == sb["sweeps"] and sa["status"] == 0
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-12 * np.abs(a).max())


def _mid_spectrum_case():
    """rhs = L of an eigenmode with Jacobi eigenvalue 1 (the fixed-weight
    sweep removes it at once) and v, the slowest mode with horizontal and
    vertical structure (the slowest the sweeps see when both uniform parts
    start exact)."""
    p = small(nx=16, ny=16, nz=16, dx=40.0, dy=40.0, dz=10.0, poisson_scheme="jacobi",
              poisson_tol=1e-10, poisson_check_every=5)
    k, j, i = np.meshgrid(np.arange(16), np.arange(16), np.arange(16), indexing="ij")
    mode = (np.cos(2 * np.pi * 4 * i / 16) * np.cos(2 * np.pi * 4 * j / 16)
            * np.cos(np.pi * 8 * (k + 0.5) / 16))
    v = np.cos(2 * np.pi * (i + 0.5) / 16) * np.cos(np.pi * (k + 0.5) / 16)
    return p, mode, v


def test_gated_guess_kept_rejected_and_capped(oracle_lib):
    """The time step's guessed solve: a guess that starts closer than the
    zero start is kept; one that starts farther is dropped (same sweeps and
    solution as the zero start); a kept guess whose sweeps reach the cap is
    dropped and the sweeps repeated from the zero start, so the solve still
    meets the tolerance and returns the zero start's solution, with both
    passes counted.  Here the right-hand side is one eigenmode that the
    fixed-weight sweep removes in a few sweeps, and the kept guess errs by
    the slowest mode the sweeps see, which decays by 1 - omega mu_min per
    sweep."""
    p, mode, v = _mid_spectrum_case()
    rhs = oracle_lib.laplacian(p, mode)
    phi0, s0 = oracle_lib.poisson(p, rhs)
    assert s0["status"] == 0 and s0["sweeps"] <= 10
    Lv = oracle_lib.laplacian(p, v)
    a = 0.5 * np.linalg.norm(rhs) / np.linalg.norm(Lv)
    good = phi0 + a * v
    slow, sk = oracle_lib.poisson(dict(p, poisson_max_sweeps=100000), rhs, guess=good, gated=True)
    assert sk["guess"] == 1 and sk["status"] == 0 and sk["sweeps"] > 200
    bad = phi0 + 4.0 * a * v
    out, sb = oracle_lib.poisson(p, rhs, guess=bad, gated=True)
    assert sb["guess"] == 2 and sb["sweeps"] == s0["sweeps"]
    np.testing.assert_array_equal(out, phi0)
    cap = 100
    out, sc = oracle_lib.poisson(dict(p, poisson_max_sweeps=cap), rhs, guess=good, gated=True)
    assert sc["guess"] == 3 and sc["status"] == 0 and sc["sweeps"] == cap + s0["sweeps"]
    assert sc["guess_sweeps"] == cap
    np.testing.assert_array_equal(out, phi0)
    # a budget (the zero start's sweep count) ends the kept guess's sweeps at
    # the first check from there on, and the zero start takes over
    budget = 2 * s0["sweeps"] + 1
    first = -(-budget // p["poisson_check_every"]) * p["poisson_check_every"]
    out, sb = oracle_lib.poisson(dict(p, poisson_max_sweeps=100000), rhs, guess=good, gated=True,
                                 budget=budget)
    assert sb["guess"] == 3 and sb["guess_sweeps"] == first
    assert sb["sweeps"] == first + s0["sweeps"] and sb["status"] == 0
    np.testing.assert_array_equal(out, phi0)


def test_chebyshev_needs_fewer_sweeps(oracle_lib):
    shape = (16, 16, 16)
    rhs = li.random_field(shape, seed=3)
    base = dict(nx=16, ny=16, nz=16, poisson_tol=1e-8)
    _, sj = oracle_lib.poisson(small(poisson_scheme="jacobi", **base), rhs)
    _, sc = oracle_lib.poisson(small(poisson_scheme="chebyshev", **base), rhs)
    assert sj["status"] == 0 and sc["status"] == 0
    assert sc["sweeps"] * 4 < sj["sweeps"]


def test_poisson_fixed_sweeps_and_zero_rhs(oracle_lib):
    p = small(nx=8, ny=8, nz=8)
    rhs = li.random_field((8, 8, 8), seed=2)
    _, st = oracle_lib.poisson(p, rhs, fixed_sweeps=7)
    assert st["sweeps"] == 7 and st["status"] == 1
    phi, st = oracle_lib.poisson(p, np.zeros((8, 8, 8)), guess=np.full((8, 8, 8), 3.0))
    assert st["sweeps"] == 0 and np.all(phi == 0.0)


def test_poisson_not_converged_flag(oracle_lib):
    p = small(nx=8, ny=8, nz=8, poisson_max_sweeps=1, poisson_check_every=1)
    _, st = oracle_lib.poisson(p, li.random_field((8, 8, 8), seed=2))
    assert st["status"] == 1 and st["sweeps"] == 1


# ---------------------------------------------- P4 advection identities

def test_quick_constant_field_divergence_free(oracle_lib):
    """A constant scalar stays constant under a velocity whose central
    divergence vanishes (w = 0, u = -d_c psi/dy, v = d_c psi/dx)."""
    for scheme in ("quick", "weno3"):
        _constant_field(oracle_lib, small(nx=12, ny=10, nz=8, advection=scheme))


def _constant_field(oracle_lib, p):
    rs = oracle_lib.reference_state(p)
    rng = np.random.default_rng(1)
    psi = rng.standard_normal((8, 10, 12)) * 50.0
    u = -(np.roll(psi, -1, 1) - np.roll(psi, 1, 1)) / (2 * p["dy"])
    v = (np.roll(psi, -1, 2) - np.roll(psi, 1, 2)) / (2 * p["dx"])
    r0 = rs["rho0"][:, None, None]
    U, V, W = r0 * u, r0 * v, np.zeros_like(u)
    assert np.abs(oracle_lib.divergence(p, U, V, W)).max() < 1e-13
    out = oracle_lib.advect(p, U, V, W, np.full_like(u, 290.0))
    assert np.abs(out).max() < 1e-11 * 290.0 * np.abs(U).max() / p["dx"]


def test_quick_flux_divergence_of_constant_equals_central_divergence(oracle_lib):
    """Face mass flux = average of the two cells, so -div(U c) = -c div_c U
    for any momentum field, including the wall rows."""
    for scheme in ("quick", "weno3"):
        p = small(nx=8, ny=6, nz=7, advection=scheme)
        rng = np.random.default_rng(2)
        U, V, W = (rng.standard_normal((7, 6, 8)) for _ in range(3))
        out = oracle_lib.advect(p, U, V, W, np.full((7, 6, 8), 3.0))
        np.testing.assert_allclose(out, -3.0 * oracle_lib.divergence(p, U, V, W), atol=1e-13)


def test_quick_upwind_coefficients(oracle_lib):
    """1D check of the face value: for U > 0 the face value at i+1/2 is
    (6 q_i + 3 q_{i+1} - q_{i-1}) / 8, reproducing quadratics exactly."""
    p = small(nx=16, ny=4, nz=4, dx=1.0)
    x = np.arange(16, dtype=float)
    q = np.broadcast_to(0.3 * x ** 2 - x + 2.0, (4, 4, 16)).copy()
    q[..., :2] = q[..., 2:4]  # keep the periodic seam out of the checked cells
    U = np.ones((4, 4, 16))
    out = oracle_lib.advect(p, U, np.zeros_like(U), np.zeros_like(U), q)
    face = lambda s: 0.3 * s ** 2 - s + 2.0
    for i in range(4, 13):
        expect = -(face(i + 0.5) - face(i - 0.5))
        assert out[0, 0, i] == pytest.approx(expect, abs=1e-12)
    out_neg = oracle_lib.advect(p, -U, np.zeros_like(U), np.zeros_like(U), q)
    for i in range(4, 13):
        assert out_neg[0, 0, i] == pytest.approx(face(i + 0.5) - face(i - 0.5), abs=1e-12)


def test_weno3_face_values(oracle_lib):
    """WENO3 reconstruction (the paper's alternative scheme): exact on
    linear data whatever the weights; at a jump it takes the smooth side
    (the upwind cell value) where QUICK overshoots by 3/8 of the jump; for
    small smooth variations its weights tend to the linear ones, giving
    (-q_{l-1} + 5 q_l + 2 q_{l+1}) / 6; and it is unit-free (scaling the
    data scales the face value)."""
    f = lambda a, b, c: oracle_lib.face_value("weno3", a, b, c)
    for a, b, c in ((1.0, 2.0, 3.0), (290.0, 289.5, 289.0), (1e-3, 1.2e-3, 1.4e-3)):
        assert f(a, b, c) == pytest.approx(b + 0.5 * (c - b), rel=1e-14, abs=1e-300)
    assert abs(f(0.0, 0.0, 1.0)) < 1e-10
    assert abs(f(1.0, 1.0, 0.0) - 1.0) < 1e-10
    assert oracle_lib.face_value("quick", 0.0, 0.0, 1.0) == pytest.approx(0.375)
    a, b, c = 290.0, 290.0 + 1e-5, 290.0 + 3e-5
    assert f(a, b, c) == pytest.approx((-a + 5 * b + 2 * c) / 6, rel=1e-13)
    rng = np.random.default_rng(9)
    for _ in range(20):
        a, b, c = rng.standard_normal(3)
        for lam in (1e-3, 1e3):
            assert f(lam * a, lam * b, lam * c) == pytest.approx(lam * f(a, b, c), rel=1e-9)


def test_weno3_lax_friedrichs_flux_is_upwind_reconstruction(oracle_lib):
    """With the face speed |m| the Lax-Friedrichs flux takes the
    reconstruction from the upwind side: reversing the velocity mirrors
    the tendency of a mirrored field."""
    p = small(nx=16, ny=4, nz=4, dx=1.0, advection="weno3")
    rng = np.random.default_rng(3)
    q = np.broadcast_to(rng.standard_normal(16), (4, 4, 16)).copy()
    U = np.full((4, 4, 16), 1.5)
    out = oracle_lib.advect(p, U, 0 * U, 0 * U, q)
    qm = q[..., ::-1].copy()
    out_m = oracle_lib.advect(p, -U, 0 * U, 0 * U, qm)
    np.testing.assert_allclose(out_m[..., ::-1], out, rtol=1e-12, atol=1e-12)
    # explicit upwind face values for U > 0
    fv = np.array([oracle_lib.face_value("weno3", q[0, 0, (i - 1) % 16], q[0, 0, i],
                                         q[0, 0, (i + 1) % 16]) for i in range(16)])
    expect = -1.5 * (fv - np.roll(fv, 1))
    np.testing.assert_allclose(out[0, 0], expect, rtol=1e-12, atol=1e-12)


# ------------------------------------------------------- P9 orders

def test_diffusion_second_order(oracle_lib):
    errs = []
    for n in (8, 16, 32):
        H = 400.0
        p = small(nx=n, ny=n, nz=n, dx=1000.0 / n, dy=1000.0 / n, dz=H / n)
        z = li.cell_heights(p)[:, None, None]
        x = ((np.arange(n) + 0.5) * p["dx"])[None, None, :]
        y = ((np.arange(n) + 0.5) * p["dy"])[None, :, None]
        a, b, c = 2 * np.pi / 1000.0, 2 * np.pi / 1000.0, np.pi / H
        q = np.sin(a * x) * np.sin(b * y) * np.cos(c * z)
        nu = np.full(q.shape, 3.0)
        out = oracle_lib.diffuse(p, nu, 1.0, q)
        rs = oracle_lib.reference_state(p)
        rho = rs["rho0"][:, None, None]
        T0 = rs["T0"][:, None, None]
        # d rho0 / dz from rho0 ~ T0^(cpd/Rd - 1), T0 = theta0 - g z / cpd
        drho = rho * (p["cpd"] / p["Rd"] - 1.0) * (-p["g"] / p["cpd"]) / T0
        lap = -(a * a + b * b + c * c) * q
        dqdz = -c * np.sin(a * x) * np.sin(b * y) * np.sin(c * z)
        exact = 3.0 * (rho * lap + drho * dqdz)
        errs.append(np.abs(out - exact).max() / np.abs(exact).max())
    assert 3.5 < errs[0] / errs[1] < 4.5 and 3.5 < errs[1] / errs[2] < 4.5, errs


def test_weno3_advection_order(oracle_lib):
    """WENO3 (Jiang-Shu weights): second order in the mean, at least second
    order away from extrema in the maximum norm (at smooth extrema the
    nonlinear weights lower it, a known property of the scheme)."""
    l1, away = [], []
    for n in (16, 32, 64):
        p = small(nx=n, ny=4, nz=4, dx=1.0 / n, dy=1.0, dz=1.0, advection="weno3")
        x = ((np.arange(n) + 0.5) / n)[None, None, :]
        q = np.broadcast_to(np.sin(2 * np.pi * x), (4, 4, n)).copy()
        U = np.full((4, 4, n), 2.0)
        err = np.abs(oracle_lib.advect(p, U, 0 * U, 0 * U, q)
                     + 2.0 * 2 * np.pi * np.cos(2 * np.pi * x))
        l1.append(err.mean())
        away.append(err[np.broadcast_to(np.abs(np.cos(2 * np.pi * x)) > 0.5, err.shape)].max())
    assert l1[0] / l1[1] > 3.6 and l1[1] / l1[2] > 3.6, l1
    assert away[0] / away[1] > 3.6 and away[1] / away[2] > 3.6, away


def test_advection_order_at_least_two(oracle_lib):
    errs = []
    for n in (16, 32, 64):
        p = small(nx=n, ny=4, nz=4, dx=1.0 / n, dy=1.0, dz=1.0)
        x = ((np.arange(n) + 0.5) / n)[None, None, :]
        q = np.broadcast_to(np.sin(2 * np.pi * x), (4, 4, n)).copy()
        U = np.full((4, 4, n), 2.0)
        out = oracle_lib.advect(p, U, 0 * U, 0 * U, q)
        exact = -2.0 * 2 * np.pi * np.cos(2 * np.pi * x)
        errs.append(np.abs(out - exact).max())
    assert errs[0] / errs[1] > 3.6 and errs[1] / errs[2] > 3.6, errs


# ------------------------------------------------ SGS viscosity pins

def test_sgs_pure_shear(oracle_lib):
    """u = s*y (periodic-safe in the interior rows): S = |s|, nu = (cs D)^2 |s|
    for neutral stratification; f_B = 0 for Ri >= Pr."""
    p = small(nx=6, ny=12, nz=6)
    s = 0.01
    y = (np.arange(12) * p["dy"])[None, :, None] * np.ones((6, 12, 6))
    u = s * y
    z0 = np.zeros_like(u)
    nu = oracle_lib.sgs_nu(p, u, z0, z0, z0)
    delta = (p["dx"] * p["dy"] * p["dz"]) ** (1 / 3)
    # interior levels: the no-slip walls add strain in the first and last rows
    np.testing.assert_allclose(nu[1:5, 2:10, :], (p["cs"] * delta) ** 2 * s, rtol=1e-13)
    # stable stratification with N^2 = Pr S^2 / 2: f_B = sqrt(1/2)
    zc = li.cell_heights(p)[:, None, None] * np.ones((6, 12, 6))
    b = 0.5 * p["Pr"] * s * s * zc
    nu2 = oracle_lib.sgs_nu(p, u, z0, z0, b)
    np.testing.assert_allclose(nu2[1:5, 2:10, :], (p["cs"] * delta) ** 2 * s * np.sqrt(0.5), rtol=1e-12)
    b3 = 2.0 * p["Pr"] * s * s * zc
    nu3 = oracle_lib.sgs_nu(p, u, z0, z0, b3)
    assert np.all(nu3[1:5, 2:10, :] == 0.0)


def test_sgs_momentum_uniform_viscosity_is_laplacian(oracle_lib):
    """For constant nu, rho0 and divergence-free periodic u, div(rho0 sigma)
    = rho0 nu times the (wide/compact mixed) Laplacian; check for a single
    Fourier mode u = sin(a y) where sigma reduces to the compact form."""
    p = small(nx=8, ny=16, nz=6, g=0.0)
    a = 2 * np.pi / 16
    j = np.arange(16)[None, :, None] * np.ones((6, 16, 8))
    u = np.sin(a * j)
    z0 = np.zeros_like(u)
    nu = np.full_like(u, 2.0)
    fx, fy, fz = oracle_lib.sgs_momentum(p, nu, u, z0, z0)
    rho = oracle_lib.reference_state(p)["rho0"]
    assert np.allclose(rho, rho[0])
    expect = rho[0] * 2.0 * (-(2 - 2 * np.cos(a)) / p["dy"] ** 2) * u
    # interior levels (the no-slip walls add wall stress in the end rows)
    np.testing.assert_allclose(fx[1:-1], expect[1:-1], atol=1e-14)
    assert np.abs(fy[1:-1]).max() < 1e-14 and np.abs(fz[1:-1]).max() < 1e-14
    # wall rows: extra drag -rho0 nu * 2 u / dz^2 from the mirrored ghost
    np.testing.assert_allclose(fx[0], expect[0] - rho[0] * 2.0 * 2.0 * u[0] / p["dz"] ** 2,
                               atol=1e-14)


# ------------------------------------------------------ radiation

def test_radiation_column_budget(oracle_lib):
    """Integrated heating sum c_pm Pi * tend * dz telescopes to
    F(bottom) - F(top) = F0 (exp(-kappa LWP) - 1)."""
    p = small("C1m", nx=4, ny=4)
    rs = oracle_lib.reference_state(p)
    rng = np.random.default_rng(4)
    ql = np.maximum(0, rng.standard_normal((p["nz"], 4, 4))) * 3e-4
    cpmpi = 1000.0 + rng.random((p["nz"], 4, 4))
    out = oracle_lib.radiation(p, ql, cpmpi)
    lwp = (rs["rho0"][:, None, None] * ql * p["dz"]).sum(axis=0)
    col = (out * cpmpi * p["dz"]).sum(axis=0)
    np.testing.assert_allclose(col, p["rad_F0"] * (np.exp(-p["rad_kappa"] * lwp) - 1.0), rtol=1e-12)


# --------------------------------------------- P5 / P6 / P11 full step

def _random_velocity(p, state, amp=1.0, seed=9):
    rng = np.random.default_rng(seed)
    for k in ("u", "v", "w"):
        state[k] = state[k] + amp * rng.standard_normal(state[k].shape)


def _masses(p, state, oracle_lib):
    d = oracle_lib.diagnostics(p, state)
    return d["mass_thl"], d["mass_qt"]


@pytest.mark.parametrize("scheme", ["quick", "weno3"])
def test_scalar_conservation_full_step(oracle_lib, scheme):
    """Sec. 2.4: domain integrals of scalars are conserved to machine
    precision without non-conservative sources (no surface flux, radiation
    or subsidence), whatever the velocity and viscosity, with either
    advection scheme."""
    p = small("C1m", nx=12, ny=10, nz=16, shf=0.0, lhf=0.0, rad_F0=0.0,
              poisson_tol=1e-6, poisson_scheme="chebyshev", advection=scheme)
    st = li.initial_state(p)
    _random_velocity(p, st)
    m0 = _masses(p, st, oracle_lib)
    for _ in range(3):
        oracle_lib.step(p, st, nsteps=1)
        m1 = _masses(p, st, oracle_lib)
        assert abs(m1[0] - m0[0]) <= 1e-14 * abs(m0[0]) * 4
        assert abs(m1[1] - m0[1]) <= 1e-14 * abs(m0[1]) * 4
    # and the state did change
    assert np.abs(st["w"]).max() > 0.1


@pytest.mark.parametrize("scheme", ["quick", "weno3"])
def test_horizontal_momentum_conservation_free_slip(oracle_lib, scheme):
    """Sec. 2.4: flux-form advection and the divergence of the SGS stress
    only move momentum between cells; nothing crosses the periodic sides, and
    free-slip walls carry neither mass flux nor stress.  The central pressure
    gradient of a periodic field sums to zero along x and y, and buoyancy
    acts on w only.  Without Coriolis, sponge and large-scale forcing the
    domain integrals of rho0 u and rho0 v are conserved to round-off by full
    steps, with the Smagorinsky viscosity varying in space.  A dropped or
    mis-signed flux term, an unmatched face value or a wrong wall parity
    breaks this (no-slip walls exert a stress, so there it must not hold)."""
    def run(wall):
        p = small("C1m", nx=12, ny=10, nz=16, fcor=0.0, ug=0.0, vg=0.0, sponge_max=0.0,
                  wall=wall, poisson_tol=1e-8, poisson_scheme="chebyshev", advection=scheme)
        st = li.initial_state(p)
        _random_velocity(p, st)
        rho0 = oracle_lib.reference_state(p)["rho0"][:, None, None]
        mom = lambda s: np.array([(rho0 * s[c]).sum() for c in ("u", "v")])
        scale = np.array([(rho0 * np.abs(st[c])).sum() for c in ("u", "v")])
        m0 = mom(st)
        drift = []
        for _ in range(3):
            oracle_lib.step(p, st, nsteps=1)
            drift.append(np.abs(mom(st) - m0) / scale)
        assert np.abs(st["w"]).max() > 0.1
        return np.max(drift)
    assert run("free_slip") <= 1e-13
    assert run("no_slip") > 1e-6


def test_surface_flux_budget(oracle_lib):
    p = small("C1m", nx=8, ny=8, nz=16, rad_F0=0.0, poisson_tol=1e-6,
              poisson_scheme="chebyshev")
    st = li.initial_state(p)
    _random_velocity(p, st, amp=0.5)
    m0 = _masses(p, st, oracle_lib)
    oracle_lib.step(p, st, nsteps=2)
    m1 = _masses(p, st, oracle_lib)
    area = p["nx"] * p["dx"] * p["ny"] * p["dy"]
    d_thl = 2 * p["dt"] * p["shf"] / p["cpd"] * area
    d_qt = 2 * p["dt"] * p["lhf"] / p["Lv0"] * area
    # exact up to round-off of the domain integral itself
    assert abs((m1[0] - m0[0]) - d_thl) <= 1e-14 * 8 * abs(m0[0])
    assert abs((m1[1] - m0[1]) - d_qt) <= 1e-14 * 8 * abs(m0[1])
    assert d_thl > 1e4 * 1e-14 * abs(m0[0])


def test_rest_state_is_bitwise_steady(oracle_lib):
    p = small(nx=8, ny=8, nz=8, ug=0.0, vg=0.0, noise_thl=0.0, thl_ml=290.0, dthl_inv=0.0,
              qt_ml=0.0, qt_ft=0.0)
    p["z_inv"] = 1e9
    st = li.initial_state(p)
    ref = {k: v.copy() for k, v in st.items()}
    recs, _ = oracle_lib.step(p, st, nsteps=3)
    for k in st:
        assert np.array_equal(st[k], ref[k]), k
    assert all(r["sweeps"] == 0 for r in recs)


# ---------------------------------------------- P10 single-column ODEs

def _column_state(p, u, v):
    st = li.initial_state(p)
    st["u"][:] = u
    st["v"][:] = v
    st["thl"][:] = p["theta0"]
    st["qt"][:] = 0.0
    return st


@pytest.mark.parametrize("K", [1, 2, 3])
def test_inertial_oscillation(oracle_lib, K):
    """c_s = 0, no sponge, horizontally uniform wind u - u_g: the scheme
    reduces to dz/dt = -i f z for z = (u - u_g) + i (v - v_g).  Each step
    multiplies z by the amplification factor of K predictor-corrector
    sub-iterations, a(x) with a_1 = 1 + x, a_{k+1} = 1 + x (1 + a_k)/2,
    x = -i f dt."""
    p = small(nx=4, ny=4, nz=8, cs=0.0, sponge_max=0.0, noise_thl=0.0, n_subiter=K,
              dt=600.0)
    st = _column_state(p, p["ug"] + 3.0, p["vg"] - 1.0)
    z0 = complex(3.0, -1.0)
    x = -1j * p["fcor"] * p["dt"]
    a = 1 + x
    for _ in range(K - 1):
        a = 1 + x * (1 + a) / 2
    nsteps = 20
    oracle_lib.step(p, st, nsteps=nsteps)
    expect = z0 * a ** nsteps
    got = (st["u"] - p["ug"]) + 1j * (st["v"] - p["vg"])
    np.testing.assert_allclose(got, expect, rtol=1e-12)
    assert np.abs(st["w"]).max() == 0.0


def test_inertial_period_converges(oracle_lib):
    """With small f dt the oscillation has period 2 pi / f."""
    p = small(nx=4, ny=4, nz=4, cs=0.0, sponge_max=0.0, noise_thl=0.0, dt=60.0)
    st = _column_state(p, p["ug"] + 1.0, p["vg"])
    period = 2 * np.pi / p["fcor"]
    n = int(round(period / p["dt"]))
    oracle_lib.step(p, st, nsteps=n)
    assert st["u"][0, 0, 0] - p["ug"] == pytest.approx(1.0, abs=2e-2)
    assert abs(st["v"][0, 0, 0] - p["vg"]) < 2e-2


def test_sponge_decay(oracle_lib):
    """f = 0: a horizontally uniform wind anomaly relaxes at rate beta(z);
    amplification per step with K = 2 is 1 - h + h^2/2, h = beta dt."""
    p = small(nx=4, ny=4, nz=40, cs=0.0, fcor=0.0, noise_thl=0.0, sponge_frac=0.2)
    st = _column_state(p, p["ug"] + 2.0, p["vg"] + 1.0)
    oracle_lib.step(p, st, nsteps=5)
    z = li.cell_heights(p)
    H = p["nz"] * p["dz"]
    zs = 0.8 * H
    beta = np.where(z >= zs, p["sponge_max"] * np.sin(0.5 * np.pi * (z - zs) / (H - zs)) ** 2, 0.0)
    h = beta * p["dt"]
    amp = (1 - h + h * h / 2) ** 5
    np.testing.assert_allclose(st["u"][:, 0, 0] - p["ug"], 2.0 * amp, rtol=1e-12)
    np.testing.assert_allclose(st["v"][:, 0, 0] - p["vg"], 1.0 * amp, rtol=1e-12)
    assert beta[-1] > 0.24 and beta[0] == 0.0


# ---------------------------------------------- projection behaviour (R16)

def test_divergence_falls_with_subiterations(oracle_lib):
    """Post-projection central divergence drops as K grows (the lagged App. A
    correction converges).  The paper gives no threshold: parity unpinned."""
    divs = []
    for K in (1, 2, 4):
        p = small(nx=12, ny=12, nz=12, n_subiter=K, poisson_tol=1e-10,
                  poisson_scheme="chebyshev")
        st = li.initial_state(p)
        _random_velocity(p, st, amp=0.5, seed=3)
        oracle_lib.step(p, st, nsteps=1)
        divs.append(oracle_lib.diagnostics(p, st)["div_l2"])
    assert divs[1] < divs[0] and divs[2] < divs[1], divs


def test_hydrostatic_adjustment_sign(oracle_lib):
    """A horizontally uniform buoyancy at rest is balanced by the pressure
    perturbation: rho0 d_c(alpha0 p')/dz = rho0 b in the interior (Sec. 2.1
    momentum equation), so p' increases with height where b > 0.  A wrong
    sign of buoyancy or of the pressure-gradient term gives ratio -1."""
    p = small(nx=4, ny=4, nz=32, n_subiter=8, noise_thl=0.0, ug=0.0, vg=0.0, cs=0.0,
              poisson_tol=1e-12, poisson_scheme="chebyshev")
    st = li.initial_state(p)
    rs = oracle_lib.reference_state(p)
    oracle_lib.step(p, st, nsteps=2)
    b = oracle_lib.thermo(p, st["thl"], st["qt"])["b"][:, 0, 0]
    assert b.min() > 0.01
    psi = rs["alpha0"] * st["p"][:, 0, 0]
    ratio = (psi[2:] - psi[:-2]) / (2 * p["dz"]) / b[1:-1]
    assert abs(ratio.mean() - 1.0) < 0.02
    assert np.all((ratio > 0.85) & (ratio < 1.15))
    assert np.abs(st["w"]).max() < 0.01


def test_radiation_cools_column(oracle_lib):
    """Radiative flux divergence (Sec. 2.1 theta_l equation) removes
    F0 (1 - exp(-kappa LWP)) / (c_pm Pi) per unit area and time."""
    p = small("C1m", nx=4, ny=4, ug=0.0, vg=0.0, shf=0.0, lhf=0.0, noise_thl=0.0,
              noise_qt=0.0, cs=0.0, poisson_tol=1e-8, poisson_scheme="chebyshev")
    st = li.initial_state(p)
    m0 = oracle_lib.diagnostics(p, st)["mass_thl"]
    th = oracle_lib.thermo(p, st["thl"], st["qt"])
    oracle_lib.step(p, st, nsteps=1)
    m1 = oracle_lib.diagnostics(p, st)["mass_thl"]
    rs = oracle_lib.reference_state(p)
    lwp = rs["rho0"] @ th["ql"][:, 0, 0] * p["dz"]
    assert lwp > 0.05
    area = p["nx"] * p["dx"] * p["ny"] * p["dy"]
    expect = p["dt"] * p["rad_F0"] * (np.exp(-p["rad_kappa"] * lwp) - 1) / p["cpd"] * area
    assert 0.95 < (m1 - m0) / expect < 1.05


# ------------------------------------------- P12 initial guesses of the solve

def test_guess_modes_change_sweeps_not_solution(oracle_lib):
    """A starting iterate only changes how many sweeps the solve takes: the
    stopping test is relative to ||rhs|| (Sec. 2.4 solve), so every guess
    ends within the tolerance-level distance of the zero-guess run, and each
    solve meets the tolerance.  Reusing the last step's solution of the same
    sub-iteration saves sweeps once the flow is past its first adjustment; a
    guess taken from the wrong sub-iteration or not gauged would not."""
    p0 = small("C1m", poisson_tol=1e-8, poisson_scheme="chebyshev")
    runs = {}
    for g in ("zero", "previous", "extrapolate"):
        p = dict(p0, guess=g)
        st = li.initial_state(p)
        recs, _ = oracle_lib.step(p, st, nsteps=10)
        for r in recs:
            assert r["status"] == 0 and r["res_norm"] <= p["poisson_tol"] * r["rhs_norm"]
        runs[g] = (st, recs)
    ref, rz = runs["zero"]
    K = p0["n_subiter"]
    for g in ("previous", "extrapolate"):
        st, recs = runs[g]
        # first step: nothing to reuse, identical solves
        assert [r["sweeps"] for r in recs[:K]] == [r["sweeps"] for r in rz[:K]]
        for k in st:
            d = ref[k] - ref[k].mean(axis=(1, 2), keepdims=True)
            assert np.linalg.norm(st[k] - ref[k]) <= 1e-6 * np.linalg.norm(d), (g, k)
    sw = lambda recs, k: sum(r["sweeps"] for i, r in enumerate(recs[4 * K:]) if i % K == k)
    st, rp = runs["previous"]
    for k in range(K):
        assert sw(rp, k) < sw(rz, k), k
    # start codes: 0 zero start, 1 guess kept, 2 guess rejected (its residual
    # not below ||rhs||); no guess exists on the first step, and once the
    # flow has passed its first adjustment the previous solution is kept
    assert all(r["guess"] == 0 for r in rz)
    assert [r["guess"] for r in rp[:K]] == [0] * K
    assert all(r["guess"] == 1 for r in rp[6 * K:])
    assert all(r["guess"] in (1, 2) for r in rp[K:])
    with pytest.raises(ValueError):
        oracle_lib.make_cfg(dict(p0, guess="learned"))


# ------------------------------- validation-case options (Sec. 3): uniform
# viscosity and free-slip walls, pinned by exact discrete decay rates

def _amp(x, K):
    """Amplification per step of K predictor-corrector sub-iterations for
    dq/dt = (x/dt) q (the recurrence of the inertial-oscillation pin)."""
    a = 1 + x
    for _ in range(K - 1):
        a = 1 + x * (1 + a) / 2
    return a


def _quiet(**kw):
    """g = 0 (uniform reference state, no buoyancy), no Coriolis, sponge,
    forcing or noise, uniform viscosity: momentum and scalars only diffuse."""
    base = dict(nx=4, ny=4, nz=16, dx=40.0, dy=40.0, dz=10.0, dt=5.0, g=0.0, fcor=0.0,
                ug=0.0, vg=0.0, sponge_max=0.0, noise_thl=0.0, nu_const=2.0,
                poisson_tol=1e-10)
    base.update(kw)
    return small(**base)


@pytest.mark.parametrize("wall", ["free_slip", "no_slip"])
def test_wall_condition_shear_mode_decay(oracle_lib, wall):
    """A horizontally uniform shear flow u(z) with w = 0 is divergence free and
    not advected, so it only diffuses.  Free slip mirrors u evenly across the
    walls, whose discrete eigenmodes are cos(pi m (k + 1/2) / nz); no slip
    mirrors it oddly, with modes sin(pi m (k + 1/2) / nz); both m = 1 modes
    have the eigenvalue -(2 - 2 cos(pi / nz)) / dz^2.  Free slip also keeps
    the column mean (zero wall stress).  A parity mistake in any stress or
    advection term changes the decay or moves the mean."""
    p = _quiet(wall=wall, nu_const=5.0)
    nz, K = p["nz"], p["n_subiter"]
    kk = np.arange(nz) + 0.5
    mode = np.cos(np.pi * kk / nz) if wall == "free_slip" else np.sin(np.pi * kk / nz)
    mean = 1.5 if wall == "free_slip" else 0.0
    st = _column_state(p, 0.0, 0.0)
    st["u"][:] = (mean + 2.0 * mode)[:, None, None]
    lam = (2 - 2 * np.cos(np.pi / nz)) / p["dz"] ** 2
    x = -p["nu_const"] * lam * p["dt"]
    nsteps = 20
    oracle_lib.step(p, st, nsteps=nsteps)
    expect = mean + 2.0 * mode * _amp(x, K) ** nsteps
    np.testing.assert_allclose(st["u"][:, 1, 2], expect, rtol=1e-12, atol=1e-13)
    assert _amp(x, K) ** nsteps < 0.9  # the decay is large enough to see
    assert np.abs(st["w"]).max() == 0.0 and np.abs(st["v"]).max() == 0.0


def test_uniform_viscosity_horizontal_modes(oracle_lib):
    """With nu uniform and free-slip walls (no-slip walls would add their
    stress to the z-uniform v), a mode cos(2 pi x / Lx) of v (divergence
    free), of theta_l and of q_t decays with the periodic eigenvalue
    -(2 - 2 cos(2 pi / nx)) / dx^2 times nu, nu / Pr and nu / Sc
    respectively (Sc set apart from Pr so a swapped number shows)."""
    p = _quiet(nx=16, nz=4, dx=10.0, dy=10.0, Sc=0.7, wall="free_slip")
    nx, K = p["nx"], p["n_subiter"]
    c = np.cos(2 * np.pi * (np.arange(nx) + 0.5) / nx)[None, None, :]
    st = _column_state(p, 0.0, 0.0)
    st["v"] = np.broadcast_to(3.0 * c, st["v"].shape).copy()
    st["thl"] = p["theta0"] + np.broadcast_to(0.5 * c, st["thl"].shape)
    st["qt"] = 1e-3 + np.broadcast_to(1e-4 * c, st["qt"].shape)
    lam = (2 - 2 * np.cos(2 * np.pi / nx)) / p["dx"] ** 2
    nsteps = 10
    oracle_lib.step(p, st, nsteps=nsteps)
    for f, base, a, kappa in (("v", 0.0, 3.0, p["nu_const"]),
                              ("thl", p["theta0"], 0.5, p["nu_const"] / p["Pr"]),
                              ("qt", 1e-3, 1e-4, p["nu_const"] / p["Sc"])):
        amp = _amp(-kappa * lam * p["dt"], K) ** nsteps
        assert amp < 0.95
        np.testing.assert_allclose(st[f] - base, a * amp * np.broadcast_to(c, st[f].shape),
                                   rtol=0, atol=abs(a) * 1e-11, err_msg=f)


def test_validation_case_parameters_match_paper():
    """The dry validation workloads carry the amplitudes, radii, domain sizes,
    viscosities, end times and resolution range that Sec. 3 prints
    (tests/golden/validation_cases.txt); their grids span the domain."""
    golden = {}
    with open(os.path.join(os.path.dirname(__file__), "golden", "validation_cases.txt")) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                case, name, value = line.split()
                golden.setdefault(case, {})[name] = float(value)
    for case, vals in golden.items():
        d = li.DRY_CASES[case]
        for name, v in vals.items():
            if name == "h_coarsest":
                assert v in li.DRY_RESOLUTIONS
            elif name == "h_finest":
                assert min(li.DRY_RESOLUTIONS) == v
            else:
                assert d[name] == v, (case, name)
        for h in li.DRY_RESOLUTIONS:
            p = li.workload(f"{case}{h}")
            assert p["nx"] * p["dx"] == vals["Lx"] and p["nz"] * p["dz"] == vals["H"]
            assert p["ny"] == 1 and p["nu_const"] == vals["nu_const"]
            assert p["bubble_amp"] == vals["bubble_amp"]


@pytest.mark.parametrize("case", ["DC400", "RB400"])
def test_validation_case_mirror_symmetry(oracle_lib, case):
    """The density-current and rising-bubble initial states are mirror
    symmetric about x = Lx/2 (a cell face), and the equations are invariant
    under x -> -x with u -> -u, so theta_l and w stay symmetric and u
    antisymmetric.  The QUICK upwind side flips with the sign of the face
    flux; a stencil oriented the same way for both signs breaks this."""
    p = small(case, precision="fp64", poisson_tol=1e-9)
    st = li.initial_state(p)
    oracle_lib.step(p, st, nsteps=4)
    t, u, w = st["thl"][:, 0, :], st["u"][:, 0, :], st["w"][:, 0, :]
    assert np.abs(w).max() > 0.1
    dev = p["theta_bg"] - t
    assert np.abs(dev - dev[:, ::-1]).max() <= 1e-12 * np.abs(dev).max()
    assert np.abs(u + u[:, ::-1]).max() <= 1e-12 * np.abs(u).max()
    assert np.abs(w - w[:, ::-1]).max() <= 1e-12 * np.abs(w).max()


@pytest.mark.parametrize("case,sign", [("DC400", -1), ("RB400", 1)])
def test_validation_case_bubble_moves_with_its_buoyancy(oracle_lib, case, sign):
    """A cold bubble starts sinking and a warm one rising: w at the bubble
    centre has the sign of the perturbation and the flow converges (cold)
    or diverges (warm) below it."""
    p = small(case, precision="fp64", poisson_tol=1e-9)
    st = li.initial_state(p)
    oracle_lib.step(p, st, nsteps=4)
    kc = int(p["bubble_zc"] / p["dz"])
    ic = p["nx"] // 2
    assert sign * st["w"][kc, 0, ic] > 0
    assert sign * st["w"][kc, 0, ic] > 0.5 * sign * st["w"][:, 0, :].max() * sign
