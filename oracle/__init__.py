"""Python access to the serial FP64 CPU oracle (oracle/les_oracle.c).

TEST INFRASTRUCTURE ONLY.  The tests, the smoke check and the benchmark's
CPU-baseline leg use it; the GPU library and its binding never import it.
Arrays are float64 numpy arrays of shape (nz, ny, nx).
"""
from __future__ import annotations

import contextlib
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

SCHEMES = {"jacobi": 0, "chebyshev": 1}


GUESSES = {"zero": 0, "extrapolate": 1, "previous": 2}
ADVECTION = {"quick": 0, "weno3": 1}
WALLS = {"no_slip": 0, "free_slip": 1}
PHASES = {"heaviside": 0, "ramp": 1}
MEAN_MODES = {"swept": 0, "level": 1, "exact": 2}


class OCfg(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("n_subiter", C.c_int32),
        ("poisson_scheme", C.c_int32), ("poisson_check_every", C.c_int32),
        ("poisson_max_sweeps", C.c_int32), ("satadj_maxit", C.c_int32),
        ("guess", C.c_int32), ("advection", C.c_int32),
        ("wall", C.c_int32), ("phase", C.c_int32), ("mean_mode", C.c_int32),
        ("reserved", C.c_int32),
        ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double), ("dt", C.c_double),
        ("poisson_tol", C.c_double), ("jacobi_omega", C.c_double),
        ("p00", C.c_double), ("theta0", C.c_double), ("Rd", C.c_double), ("Rv", C.c_double),
        ("cpd", C.c_double), ("cpv", C.c_double), ("cl", C.c_double), ("ci", C.c_double),
        ("Lv0", C.c_double), ("Ls0", C.c_double), ("Tf", C.c_double), ("fcor", C.c_double),
        ("g", C.c_double), ("cs", C.c_double), ("Pr", C.c_double), ("Sc", C.c_double),
        ("ug", C.c_double), ("vg", C.c_double), ("shf", C.c_double), ("lhf", C.c_double),
        ("wsub_div", C.c_double), ("sponge_frac", C.c_double), ("sponge_max", C.c_double),
        ("rad_F0", C.c_double), ("rad_kappa", C.c_double),
        ("e_tr", C.c_double), ("T_tr", C.c_double), ("satadj_tol", C.c_double),
        ("nu_const", C.c_double), ("T_ice", C.c_double),
    ]


class OSolve(C.Structure):
    _fields_ = [("sweeps", C.c_int32), ("status", C.c_int32),
                ("rhs_norm", C.c_double), ("res_norm", C.c_double),
                ("guess", C.c_int32), ("guess_sweeps", C.c_int32)]


class ODebug(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in ("b_half", "nu", "rhs", "phi", "uhat", "vhat", "what")]


_lib = None
_DP = C.POINTER(C.c_double)


def _bind(L):
    """Set the ctypes signatures of an oracle library."""
    cfgp = C.POINTER(OCfg)
    L.oracle_reference_state.argtypes = [cfgp, _DP, _DP, _DP, _DP]
    L.oracle_exner.argtypes = [cfgp] + [C.c_double] * 4
    L.oracle_exner.restype = C.c_double
    L.oracle_theta_l.argtypes = [cfgp] + [C.c_double] * 5
    L.oracle_theta_l.restype = C.c_double
    L.oracle_qv_sat.argtypes = [cfgp, C.c_double, C.c_double]
    L.oracle_qv_sat.restype = C.c_double
    for name in ("oracle_qv_sat_ice", "oracle_qv_star"):
        getattr(L, name).argtypes = [cfgp, C.c_double, C.c_double]
        getattr(L, name).restype = C.c_double
    L.oracle_liquid_fraction.argtypes = [cfgp, C.c_double]
    L.oracle_liquid_fraction.restype = C.c_double
    L.oracle_satadj.argtypes = [cfgp, C.c_double, C.c_double, C.c_double, _DP, _DP, _DP]
    L.oracle_thermo.argtypes = [cfgp, _DP, _DP, _DP, _DP, _DP, _DP]
    L.oracle_sgs_nu.argtypes = [cfgp, _DP, _DP, _DP, _DP, _DP]
    L.oracle_advect.argtypes = [cfgp, _DP, _DP, _DP, _DP, C.c_double, _DP]
    L.oracle_face_value.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double]
    L.oracle_face_value.restype = C.c_double
    L.oracle_diffuse.argtypes = [cfgp, _DP, C.c_double, _DP, _DP]
    L.oracle_sgs_momentum.argtypes = [cfgp, _DP, _DP, _DP, _DP, _DP, _DP, _DP]
    L.oracle_laplacian.argtypes = [cfgp, _DP, _DP]
    L.oracle_app_a.argtypes = [cfgp, _DP, _DP]
    L.oracle_divergence.argtypes = [cfgp, _DP, _DP, _DP, _DP]
    L.oracle_radiation.argtypes = [cfgp, _DP, _DP, _DP]
    L.oracle_poisson.argtypes = [cfgp, _DP, _DP, C.c_int32, C.POINTER(OSolve)]
    L.oracle_poisson_gated.argtypes = [cfgp, _DP, _DP, C.c_int32, C.c_int32, C.POINTER(OSolve)]
    L.oracle_jacobi_bounds.argtypes = [cfgp, _DP, _DP]
    L.oracle_vertical_mode_solve.argtypes = [cfgp, _DP, _DP]
    L.oracle_step.argtypes = [cfgp, _DP, _DP, _DP, _DP, _DP, _DP, C.c_int32,
                              C.POINTER(C.c_int32), C.POINTER(OSolve), C.POINTER(ODebug)]
    L.oracle_diagnostics.argtypes = [cfgp, _DP, _DP, _DP, _DP, _DP, _DP, _DP]
    return L


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        _lib = _bind(C.CDLL(LIB_PATH))
    return _lib


@contextlib.contextmanager
def variant(path):
    """Route every call of this module to another build of the oracle (a
    copy with a deliberately planted mistake, built by the tests to show
    that a pin fails on it) for the duration of the block."""
    global _lib
    saved = lib()
    _lib = _bind(C.CDLL(path))
    try:
        yield
    finally:
        _lib = saved


def make_cfg(p: dict) -> OCfg:
    """Oracle configuration from a full workload parameter dict."""
    c = OCfg()
    for name, ctype in OCfg._fields_:
        if name == "poisson_scheme":
            v = p["poisson_scheme"]
            c.poisson_scheme = SCHEMES[v] if isinstance(v, str) else int(v)
        elif name == "guess":
            v = p.get("guess", "zero")
            if v not in GUESSES:
                raise ValueError(f"the oracle step has no {v!r} guess; known: {sorted(GUESSES)}")
            c.guess = GUESSES[v]
        elif name == "advection":
            v = p.get("advection", "quick")
            if v not in ADVECTION:
                raise ValueError(f"unknown advection scheme {v!r}; known: {sorted(ADVECTION)}")
            c.advection = ADVECTION[v]
        elif name == "wall":
            v = p.get("wall", "no_slip")
            if v not in WALLS:
                raise ValueError(f"unknown wall condition {v!r}; known: {sorted(WALLS)}")
            c.wall = WALLS[v]
        elif name == "phase":
            v = p.get("phase", "heaviside")
            if v not in PHASES:
                raise ValueError(f"unknown phase partition {v!r}; known: {sorted(PHASES)}")
            c.phase = PHASES[v]
        elif name == "mean_mode":
            v = p.get("mean_mode", "exact")
            if v not in MEAN_MODES:
                raise ValueError(f"unknown mean mode {v!r}; known: {sorted(MEAN_MODES)}")
            c.mean_mode = MEAN_MODES[v]
        elif name == "reserved":
            c.reserved = 0
        else:
            setattr(c, name, ctype(p[name]).value)
    return c


def _ptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_DP)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")


def _shape(p):
    return (p["nz"], p["ny"], p["nx"])


def reference_state(p):
    c = make_cfg(p)
    out = [np.zeros(p["nz"]) for _ in range(4)]
    _check(lib().oracle_reference_state(C.byref(c), *[_ptr(a) for a in out]), "reference_state")
    return dict(zip(("p0", "T0", "rho0", "alpha0"), out))


def exner(p, p0, qt, ql, qi):
    return lib().oracle_exner(C.byref(make_cfg(p)), p0, qt, ql, qi)


def theta_l(p, T, ql, qi, qt, p0):
    return lib().oracle_theta_l(C.byref(make_cfg(p)), T, ql, qi, qt, p0)


def qv_sat(p, T, p0):
    return lib().oracle_qv_sat(C.byref(make_cfg(p)), T, p0)


def qv_sat_ice(p, T, p0):
    return lib().oracle_qv_sat_ice(C.byref(make_cfg(p)), T, p0)


def qv_star(p, T, p0):
    return lib().oracle_qv_star(C.byref(make_cfg(p)), T, p0)


def liquid_fraction(p, T):
    return lib().oracle_liquid_fraction(C.byref(make_cfg(p)), T)


def satadj(p, thl, qt, p0):
    T, ql, qi = C.c_double(), C.c_double(), C.c_double()
    it = lib().oracle_satadj(C.byref(make_cfg(p)), thl, qt, p0, C.byref(T), C.byref(ql), C.byref(qi))
    return T.value, ql.value, qi.value, it


def thermo(p, thl, qt):
    thl, qt = _f64(thl), _f64(qt)
    out = [np.zeros(_shape(p)) for _ in range(4)]
    _check(lib().oracle_thermo(C.byref(make_cfg(p)), _ptr(thl), _ptr(qt), *[_ptr(a) for a in out]), "thermo")
    return dict(zip(("T", "ql", "qi", "b"), out))


def sgs_nu(p, u, v, w, b):
    u, v, w, b = map(_f64, (u, v, w, b))
    nu = np.zeros(_shape(p))
    _check(lib().oracle_sgs_nu(C.byref(make_cfg(p)), _ptr(u), _ptr(v), _ptr(w), _ptr(b), _ptr(nu)), "sgs_nu")
    return nu


def face_value(scheme, qm1, q0, q1):
    """Upwind face value at l+1/2 from (q_{l-1}, q_l, q_{l+1})."""
    return lib().oracle_face_value(ADVECTION[scheme], qm1, q0, q1)


def advect(p, U, V, W, q, zparity=1.0):
    U, V, W, q = map(_f64, (U, V, W, q))
    out = np.zeros(_shape(p))
    _check(lib().oracle_advect(C.byref(make_cfg(p)), _ptr(U), _ptr(V), _ptr(W), _ptr(q),
                               float(zparity), _ptr(out)), "advect")
    return out


def diffuse(p, nu, inv_prandtl, q):
    nu, q = _f64(nu), _f64(q)
    out = np.zeros(_shape(p))
    _check(lib().oracle_diffuse(C.byref(make_cfg(p)), _ptr(nu), float(inv_prandtl), _ptr(q), _ptr(out)), "diffuse")
    return out


def sgs_momentum(p, nu, u, v, w):
    nu, u, v, w = map(_f64, (nu, u, v, w))
    out = [np.zeros(_shape(p)) for _ in range(3)]
    _check(lib().oracle_sgs_momentum(C.byref(make_cfg(p)), _ptr(nu), _ptr(u), _ptr(v), _ptr(w),
                                     *[_ptr(a) for a in out]), "sgs_momentum")
    return out


def _unary(name, p, a):
    a = _f64(a)
    out = np.zeros(_shape(p))
    _check(getattr(lib(), name)(C.byref(make_cfg(p)), _ptr(a), _ptr(out)), name)
    return out


def laplacian(p, phi):
    return _unary("oracle_laplacian", p, phi)


def app_a(p, phi):
    return _unary("oracle_app_a", p, phi)


def divergence(p, U, V, W):
    U, V, W = map(_f64, (U, V, W))
    out = np.zeros(_shape(p))
    _check(lib().oracle_divergence(C.byref(make_cfg(p)), _ptr(U), _ptr(V), _ptr(W), _ptr(out)), "divergence")
    return out


def radiation(p, ql, cpmpi):
    ql, cpmpi = _f64(ql), _f64(cpmpi)
    out = np.zeros(_shape(p))
    _check(lib().oracle_radiation(C.byref(make_cfg(p)), _ptr(ql), _ptr(cpmpi), _ptr(out)), "radiation")
    return out


def vertical_mode_solve(p, rv):
    """Solution pv (ny, nx) of the vertically uniform part Lh pv = rv."""
    rv = _f64(rv)
    assert rv.shape == (p["ny"], p["nx"])
    pv = np.zeros_like(rv)
    _check(lib().oracle_vertical_mode_solve(C.byref(make_cfg(p)), _ptr(rv), _ptr(pv)),
           "vertical_mode_solve")
    return pv


def jacobi_bounds(p):
    a, b = C.c_double(), C.c_double()
    _check(lib().oracle_jacobi_bounds(C.byref(make_cfg(p)), C.byref(a), C.byref(b)), "jacobi_bounds")
    return a.value, b.value


def poisson(p, rhs, guess=None, fixed_sweeps=0, gated=False, budget=0):
    """Returns (phi, stats dict).  gated: the solve as the time step runs it
    for a guess (kept only if it starts closer than the zero start, solved
    again from the zero start if its sweeps reach the cap or, budget > 0,
    that many sweeps)."""
    rhs = _f64(rhs)
    phi = np.zeros(_shape(p)) if guess is None else _f64(guess).copy()
    st = OSolve()
    if gated:
        rc = lib().oracle_poisson_gated(C.byref(make_cfg(p)), _ptr(rhs), _ptr(phi),
                                        int(fixed_sweeps), int(budget), C.byref(st))
    else:
        rc = lib().oracle_poisson(C.byref(make_cfg(p)), _ptr(rhs), _ptr(phi), int(fixed_sweeps),
                                  C.byref(st))
    if rc not in (0, -3):
        raise RuntimeError(f"oracle poisson failed with code {rc}")
    return phi, dict(sweeps=st.sweeps, status=st.status, rhs_norm=st.rhs_norm, res_norm=st.res_norm,
                     guess=st.guess, guess_sweeps=st.guess_sweeps)


DEBUG_FIELDS = ("b_half", "nu", "rhs", "phi", "uhat", "vhat", "what")


def step(p, state, nsteps=1, replay=None, debug=False):
    """Advance `state` (dict of u, v, w, thl, qt, p float64 arrays) in place.

    Returns (records, debug_dict): one record per Poisson solve.
    """
    c = make_cfg(p)
    arrs = [state[k] for k in ("u", "v", "w", "thl", "qt", "p")]
    for a in arrs:
        assert a.dtype == np.float64 and a.flags.c_contiguous and a.shape == _shape(p)
    nsolve = nsteps * p["n_subiter"]
    rec = (OSolve * nsolve)()
    rp = None
    if replay is not None:
        rl = np.ascontiguousarray(replay, dtype=np.int32)
        assert rl.size >= nsolve
        rp = rl.ctypes.data_as(C.POINTER(C.c_int32))
    dbg = None
    dbg_arrays = {}
    if debug:
        dbg = ODebug()
        for k in DEBUG_FIELDS:
            dbg_arrays[k] = np.zeros(_shape(p))
            setattr(dbg, k, dbg_arrays[k].ctypes.data)
    rc = lib().oracle_step(C.byref(c), *[_ptr(a) for a in arrs], int(nsteps), rp, rec,
                           C.byref(dbg) if dbg is not None else None)
    recs = [dict(sweeps=r.sweeps, status=r.status, rhs_norm=r.rhs_norm, res_norm=r.res_norm,
                 guess=r.guess, guess_sweeps=r.guess_sweeps) for r in rec]
    if rc != 0:
        raise RuntimeError(f"oracle step failed with code {rc}; solves: {recs}")
    return recs, dbg_arrays


def diagnostics(p, state):
    c = make_cfg(p)
    arrs = [_f64(state[k]) for k in ("u", "v", "w", "thl", "qt")]
    sc = np.zeros(6)
    prof = np.zeros((9, p["nz"]))
    _check(lib().oracle_diagnostics(C.byref(c), *[_ptr(a) for a in arrs], _ptr(sc), _ptr(prof)),
           "diagnostics")
    names = ("thl", "qt", "ql", "u", "v", "w", "w2", "w3", "b")
    return dict(mass_thl=sc[0], mass_qt=sc[1], div_l2=sc[2], div_max=sc[3], cfl=sc[4], ke=sc[5],
                profiles=dict(zip(names, prof)))
