"""ctypes binding of the HIP LES library (include/les.h).

Argument marshalling only: every step of the time step runs in the HIP
kernels of liblesmi.so.  PyTorch provides device memory and the stream.
The library must be built (paper_2301_04698_amd/build.py); loading fails
loudly if it is missing or does not load, and there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_lib", "liblesmi.so")

LES_OK, LES_WARN_NOT_CONVERGED = 0, 1
LES_ERR_ARG, LES_ERR_HIP, LES_ERR_NONFINITE, LES_ERR_STATE = -1, -2, -3, -4
LES_FP64, LES_FP32 = 0, 1
LES_JACOBI, LES_CHEBYSHEV = 0, 1
LES_QUICK, LES_WENO3 = 0, 1
ADVECTION = {"quick": LES_QUICK, "weno3": LES_WENO3}
LES_NO_SLIP, LES_FREE_SLIP = 0, 1
WALLS = {"no_slip": LES_NO_SLIP, "free_slip": LES_FREE_SLIP}
LES_PHASE_HEAVISIDE, LES_PHASE_RAMP = 0, 1
PHASES = {"heaviside": LES_PHASE_HEAVISIDE, "ramp": LES_PHASE_RAMP}
LES_MEAN_SWEPT, LES_MEAN_LEVEL, LES_MEAN_EXACT = 0, 1, 2
MEAN_MODES = {"swept": LES_MEAN_SWEPT, "level": LES_MEAN_LEVEL, "exact": LES_MEAN_EXACT}
LES_GUESS_ZERO, LES_GUESS_EXTRAPOLATE, LES_GUESS_PREVIOUS, LES_GUESS_LEARNED = 0, 1, 2, 3
LES_GUESS_LEARNED3 = 4
GUESS_MODES = {"zero": LES_GUESS_ZERO, "extrapolate": LES_GUESS_EXTRAPOLATE,
               "previous": LES_GUESS_PREVIOUS, "learned": LES_GUESS_LEARNED,
               "learned3": LES_GUESS_LEARNED3}
NPROFILES = 9
PROFILE_NAMES = ("thl", "qt", "ql", "u", "v", "w", "w2", "w3", "b")

# Workspace field ids (les_workspace_offset).
WS_FIELDS = ("un", "vn", "wn", "thl_half", "qt_half", "thl_mid", "qt_mid", "uh", "vh", "wh",
             "b_half", "b_mid", "ql_mid", "cpmpi_mid", "nu_s", "nu_m", "rad", "rhs", "phi0", "phi1",
             "phi2", "phi3", "p_prev", "guess", "rhs_defect")

EXPORTS = ("les_default_config", "les_workspace_bytes", "les_workspace_offset", "les_init",
           "les_step", "les_poisson_solve", "les_pressure", "les_set_pressure_profile",
           "les_thermo", "les_diagnostics", "les_state_bytes", "les_export_state",
           "les_import_state", "les_steps_done", "les_destroy", "les_last_error")


class LesConfig(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("precision", C.c_int32),
        ("n_subiter", C.c_int32), ("poisson_scheme", C.c_int32),
        ("poisson_check_every", C.c_int32), ("poisson_max_sweeps", C.c_int32),
        ("satadj_maxit", C.c_int32), ("sweeps_per_launch", C.c_int32),
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
        ("guess", C.c_int32), ("advection", C.c_int32),
        ("wall", C.c_int32), ("phase", C.c_int32), ("nu_const", C.c_double),
        ("T_ice", C.c_double), ("mean_mode", C.c_int32), ("guess_passes", C.c_int32),
    ]


class LesBuffers(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in ("u", "v", "w", "thl", "qt", "p", "workspace")] + [
        ("workspace_bytes", C.c_size_t)]


class LesSolveStats(C.Structure):
    _fields_ = [("sweeps", C.c_int32), ("status", C.c_int32), ("rhs_norm", C.c_double),
                ("res_norm", C.c_double), ("seconds", C.c_double), ("guess", C.c_int32),
                ("guess_sweeps", C.c_int32)]

    def as_dict(self):
        return dict(sweeps=self.sweeps, status=self.status, rhs_norm=self.rhs_norm,
                    res_norm=self.res_norm, seconds=self.seconds, guess=self.guess,
                    guess_sweeps=self.guess_sweeps)


class LesPoissonOpts(C.Structure):
    _fields_ = [("fixed_sweeps", C.c_int32), ("use_guess", C.c_int32), ("budget", C.c_int32)]


class LesStepOpts(C.Structure):
    _fields_ = [("replay_sweeps", C.POINTER(C.c_int32)), ("records", C.POINTER(LesSolveStats)),
                ("time_sweeps", C.c_int32), ("reserved", C.c_int32),
                ("dump_rhs", C.c_void_p), ("dump_phi", C.c_void_p),
                ("dump_mean", C.POINTER(C.c_double)), ("dump_base", C.c_void_p)]


class LesStepStats(C.Structure):
    _fields_ = [("steps", C.c_int32), ("solves", C.c_int32), ("sweeps_total", C.c_int64),
                ("sweeps_max", C.c_int32), ("not_converged", C.c_int32),
                ("res_rel_max", C.c_double), ("seconds", C.c_double),
                ("poisson_seconds", C.c_double), ("sweep_seconds", C.c_double),
                ("sweeps_timed", C.c_int64)]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


class LesDiag(C.Structure):
    _fields_ = [(n, C.c_double) for n in ("mass_thl", "mass_qt", "div_l2", "div_max", "cfl", "ke")]


class LesError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"LES error {code}: {msg}")
        self.code = code


_lib = None


def load():
    """Load liblesmi.so (building it first if it was never built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        from . import build as _b
        _b.build()
    L = C.CDLL(LIB_PATH)
    cp = C.POINTER(LesConfig)
    L.les_default_config.argtypes = [cp]
    L.les_default_config.restype = None
    L.les_workspace_bytes.argtypes = [cp]
    L.les_workspace_bytes.restype = C.c_size_t
    L.les_workspace_offset.argtypes = [cp, C.c_int32, C.POINTER(C.c_size_t)]
    L.les_init.argtypes = [cp, C.POINTER(LesBuffers), C.c_void_p, C.POINTER(C.c_void_p)]
    L.les_step.argtypes = [C.c_void_p, C.c_int32, C.POINTER(LesStepOpts), C.POINTER(LesStepStats)]
    L.les_poisson_solve.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(LesPoissonOpts),
                                    C.POINTER(LesSolveStats)]
    L.les_pressure.argtypes = [C.c_void_p, C.c_void_p, C.POINTER(C.c_double)]
    L.les_set_pressure_profile.argtypes = [C.c_void_p, C.POINTER(C.c_double)]
    L.les_state_bytes.argtypes = [C.c_void_p]
    L.les_state_bytes.restype = C.c_size_t
    L.les_export_state.argtypes = [C.c_void_p, C.c_void_p]
    L.les_import_state.argtypes = [C.c_void_p, C.c_void_p]
    L.les_steps_done.argtypes = [C.c_void_p]
    L.les_steps_done.restype = C.c_int64
    L.les_thermo.argtypes = [C.c_void_p] + [C.c_void_p] * 5
    L.les_diagnostics.argtypes = [C.c_void_p, C.POINTER(LesDiag), C.POINTER(C.c_double)]
    L.les_destroy.argtypes = [C.c_void_p]
    L.les_destroy.restype = None
    L.les_last_error.argtypes = []
    L.les_last_error.restype = C.c_char_p
    _lib = L
    return L


def last_error() -> str:
    return load().les_last_error().decode()


def check(rc, allow_warn=True):
    if rc == LES_OK or (allow_warn and rc == LES_WARN_NOT_CONVERGED):
        return rc
    raise LesError(rc, last_error())


def default_config() -> LesConfig:
    c = LesConfig()
    load().les_default_config(C.byref(c))
    return c


def make_config(p: dict) -> LesConfig:
    """les_config from a full workload parameter dict."""
    c = default_config()
    for name, ctype in LesConfig._fields_:
        if name == "sweeps_per_launch":
            c.sweeps_per_launch = int(p.get("sweeps_per_launch", 0))
        elif name == "advection":
            v = p.get("advection", "quick")
            c.advection = ADVECTION[v] if isinstance(v, str) else int(v)
        elif name == "wall":
            v = p.get("wall", "no_slip")
            c.wall = WALLS[v] if isinstance(v, str) else int(v)
        elif name == "phase":
            v = p.get("phase", "heaviside")
            c.phase = PHASES[v] if isinstance(v, str) else int(v)
        elif name == "guess":
            v = p.get("guess", "zero")
            c.guess = GUESS_MODES[v] if isinstance(v, str) else int(v)
        elif name == "mean_mode":
            v = p.get("mean_mode", "exact")
            c.mean_mode = MEAN_MODES[v] if isinstance(v, str) else int(v)
        elif name == "guess_passes":
            c.guess_passes = int(p.get("guess_passes", 0))
        elif name == "precision":
            v = p.get("precision", "fp64")
            c.precision = {"fp64": LES_FP64, "fp32": LES_FP32}[v] if isinstance(v, str) else int(v)
        elif name == "poisson_scheme":
            v = p["poisson_scheme"]
            c.poisson_scheme = {"jacobi": LES_JACOBI, "chebyshev": LES_CHEBYSHEV}[v] \
                if isinstance(v, str) else int(v)
        else:
            setattr(c, name, ctype(p[name]).value)
    return c


def workspace_bytes(cfg: LesConfig) -> int:
    return int(load().les_workspace_bytes(C.byref(cfg)))


def workspace_offset(cfg: LesConfig, field) -> int:
    fid = WS_FIELDS.index(field) if isinstance(field, str) else int(field)
    off = C.c_size_t()
    check(load().les_workspace_offset(C.byref(cfg), fid, C.byref(off)))
    return int(off.value)


class LES:
    """A simulation whose state lives in torch tensors on the current GPU."""

    def __init__(self, params: dict, state: dict | None = None, device="cuda", pbar=None):
        """state: initial u, v, w, thl, qt, p (numpy or torch); pbar: the FP64
        horizontally uniform pressure that p is relative to (exact mean
        mode; les_set_pressure_profile), default zero."""
        import torch
        self.torch = torch
        self.params = dict(params)
        self.cfg = make_config(params)
        self.dtype = torch.float64 if self.cfg.precision == LES_FP64 else torch.float32
        shape = (self.cfg.nz, self.cfg.ny, self.cfg.nx)
        self.shape = shape
        self.device = torch.device(device)
        self.fields = {}
        for k in ("u", "v", "w", "thl", "qt", "p"):
            if state is not None:
                src = state[k]
                if isinstance(src, np.ndarray):
                    src = torch.from_numpy(np.ascontiguousarray(src))
                t = src.to(device=self.device, dtype=self.dtype).contiguous().clone()
            else:
                t = torch.zeros(shape, device=self.device, dtype=self.dtype)
            assert tuple(t.shape) == shape
            self.fields[k] = t
        nbytes = workspace_bytes(self.cfg)
        if nbytes == 0:
            raise LesError(LES_ERR_ARG, last_error())
        self.workspace = torch.empty(nbytes, device=self.device, dtype=torch.uint8)
        self.bufs = LesBuffers(
            *[self.fields[k].data_ptr() for k in ("u", "v", "w", "thl", "qt", "p")],
            self.workspace.data_ptr(), nbytes)
        self.stream = torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        check(load().les_init(C.byref(self.cfg), C.byref(self.bufs), C.c_void_p(self.stream.cuda_stream),
                              C.byref(h)), allow_warn=False)
        self.handle = h
        if pbar is not None:
            pb = np.ascontiguousarray(pbar, dtype=np.float64)
            assert pb.shape == (self.cfg.nz,)
            check(load().les_set_pressure_profile(self.handle,
                                                  pb.ctypes.data_as(C.POINTER(C.c_double))),
                  allow_warn=False)

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            load().les_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _n(self):
        return self.cfg.nx * self.cfg.ny * self.cfg.nz

    def step(self, nsteps=1, replay=None, records=False, time_sweeps=False, dump=None,
             dump_mean=None, dump_base=None):
        """Advance nsteps; returns (rc, stats dict, per-solve records or None).

        dump: optional (rhs, phi) device tensors of n_subiter * n elements
        receiving the right-hand sides the last step's sweeps solved and
        their zero-mean solutions (sub-iteration k at offset k * n); with the
        exact mean mode both lack their horizontally uniform parts, which
        dump_mean (a float64 numpy array of n_subiter * (2 nz + 1) values)
        receives: per solve the per-level values the centring subtracted,
        the solution's horizontally uniform part, and the rhs mean.
        dump_base: device tensor of n_subiter * n elements receiving the
        field each of the last step's solves started its guess from."""
        K = self.cfg.n_subiter
        opts = LesStepOpts()
        opts.time_sweeps = 1 if time_sweeps else 0
        if dump is not None:
            for t in dump:
                assert t.is_contiguous() and t.dtype == self.dtype and t.numel() == K * self._n()
            opts.dump_rhs = dump[0].data_ptr()
            opts.dump_phi = dump[1].data_ptr()
        if dump_base is not None:
            assert (dump_base.is_contiguous() and dump_base.dtype == self.dtype
                    and dump_base.numel() == K * self._n())
            opts.dump_base = dump_base.data_ptr()
        if dump_mean is not None:
            assert dump_mean.dtype == np.float64 and dump_mean.flags.c_contiguous
            assert dump_mean.size == K * (2 * self.cfg.nz + 1)
            opts.dump_mean = dump_mean.ctypes.data_as(C.POINTER(C.c_double))
        rec = None
        keep = []
        if replay is not None:
            arr = np.ascontiguousarray(replay, dtype=np.int32)
            if arr.size < nsteps * K:
                raise ValueError("replay needs nsteps * n_subiter entries")
            keep.append(arr)
            opts.replay_sweeps = arr.ctypes.data_as(C.POINTER(C.c_int32))
        if records:
            rec = (LesSolveStats * (nsteps * K))()
            opts.records = C.cast(rec, C.POINTER(LesSolveStats))
        st = LesStepStats()
        rc = check(load().les_step(self.handle, int(nsteps), C.byref(opts), C.byref(st)))
        recs = [r.as_dict() for r in rec] if rec is not None else None
        return rc, st.as_dict(), recs

    def poisson_solve(self, rhs, phi=None, fixed_sweeps=0, use_guess=False, budget=0):
        """use_guess: False (zero start), True (phi holds a guess, kept) or 2
        (phi holds a guess, gated as in the time step, with a sweep budget)."""
        torch = self.torch
        rhs = rhs.to(device=self.device, dtype=self.dtype).contiguous()
        if phi is None:
            phi = torch.zeros_like(rhs)
        assert phi.is_contiguous() and phi.dtype == self.dtype and phi.numel() == self._n()
        assert rhs.numel() == self._n()
        opts = LesPoissonOpts(int(fixed_sweeps), int(use_guess), int(budget))
        st = LesSolveStats()
        rc = check(load().les_poisson_solve(self.handle, C.c_void_p(rhs.data_ptr()),
                                            C.c_void_p(phi.data_ptr()), C.byref(opts), C.byref(st)))
        return phi, st.as_dict(), rc

    def thermo(self, thl, qt):
        torch = self.torch
        thl = thl.to(device=self.device, dtype=self.dtype).contiguous()
        qt = qt.to(device=self.device, dtype=self.dtype).contiguous()
        assert thl.numel() == self._n() and qt.numel() == self._n()
        T, ql, b = (torch.empty_like(thl) for _ in range(3))
        check(load().les_thermo(self.handle, C.c_void_p(thl.data_ptr()), C.c_void_p(qt.data_ptr()),
                                C.c_void_p(T.data_ptr()), C.c_void_p(ql.data_ptr()),
                                C.c_void_p(b.data_ptr())))
        return dict(T=T, ql=ql, b=b)

    def diagnostics(self):
        d = LesDiag()
        prof = np.zeros((NPROFILES, self.cfg.nz))
        check(load().les_diagnostics(self.handle, C.byref(d),
                                     prof.ctypes.data_as(C.POINTER(C.c_double))))
        out = {n: getattr(d, n) for n, _ in LesDiag._fields_}
        out["profiles"] = dict(zip(PROFILE_NAMES, prof))
        return out

    def export_state(self):
        """The library-held state (les_export_state) as a device uint8 tensor."""
        n = int(load().les_state_bytes(self.handle))
        buf = self.torch.empty(n, dtype=self.torch.uint8, device=self.device)
        check(load().les_export_state(self.handle, C.c_void_p(buf.data_ptr())), allow_warn=False)
        return buf

    def import_state(self, buf):
        check(load().les_import_state(self.handle, C.c_void_p(buf.data_ptr())), allow_warn=False)

    def steps_done(self):
        return int(load().les_steps_done(self.handle))

    def workspace_field(self, name):
        """View of an intermediate field inside the workspace (debugging)."""
        off = workspace_offset(self.cfg, name)
        es = 8 if self.cfg.precision == LES_FP64 else 4
        raw = self.workspace[off: off + self._n() * es]
        return raw.view(self.dtype).view(self.shape)

    def pressure(self):
        """(whole p' as a device tensor, the FP64 profile kept apart)."""
        out = self.torch.empty_like(self.fields["p"])
        pbar = np.zeros(self.cfg.nz)
        check(load().les_pressure(self.handle, C.c_void_p(out.data_ptr()),
                                  pbar.ctypes.data_as(C.POINTER(C.c_double))))
        return out, pbar

    def state_split(self):
        """(state as float64 numpy arrays with p as stored, i.e. relative to
        the FP64 profile, that profile): a restart keeps p in its own
        precision and the profile in FP64."""
        self.torch.cuda.synchronize(self.device)
        out = {k: v.detach().to("cpu", dtype=self.torch.float64).numpy().copy()
               for k, v in self.fields.items()}
        return out, self.pressure()[1]

    def state_numpy(self):
        """State as float64 numpy arrays; p is the whole p' (les_pressure)."""
        self.torch.cuda.synchronize(self.device)
        out = {k: v.detach().to("cpu", dtype=self.torch.float64).numpy().copy()
               for k, v in self.fields.items()}
        out["p"] = self.pressure()[0].to("cpu", dtype=self.torch.float64).numpy()
        return out
