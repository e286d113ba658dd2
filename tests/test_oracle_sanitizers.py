"""Host sanitizer build of the FP64 oracle: the oracle's C sources and a
standalone driver (tests/sanitize_driver.c) compiled with AddressSanitizer
(leak detection on) and UndefinedBehaviorSanitizer, every report fatal.
The driver runs full-physics time steps (two configurations: warm cloud with
QUICK, no-slip walls, the exact mean modes and the previous-solution guess;
mixed-phase ice with WENO3, free slip, the level mode and the extrapolated
guess), the diagnostics of the final state, and a forward, loss and backward
pass of the guess network (one- and three-input, valid and periodic
padding); the results must equal those of the ordinary build."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import les_inputs as li

HERE = os.path.dirname(os.path.abspath(__file__))
ORACLE = os.path.join(HERE, "..", "oracle")
FIELDS = ("u", "v", "w", "thl", "qt", "p")
FLAGS = ["-O1", "-g", "-std=c11", "-fno-omit-frame-pointer", "-ffp-contract=off",
         "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-static-libasan"]


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if shutil.which("gcc") is None:
        pytest.skip("no gcc")
    d = tmp_path_factory.mktemp("sanitize")
    exe = str(d / "oracle_sanitized")
    cmd = ["gcc", *FLAGS, "-I", ORACLE, os.path.join(HERE, "sanitize_driver.c"),
           os.path.join(ORACLE, "les_oracle.c"), os.path.join(ORACLE, "cnn_oracle.c"), "-lm",
           "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and "sanitize" in r.stderr and "cannot find" in r.stderr:
        pytest.skip("the sanitizer runtimes are not installed")
    assert r.returncode == 0, r.stderr
    return exe, d


def _run(driver, p, st, nsteps, params, x, target, periodic, alpha=0.1):
    import ctypes as C
    import oracle
    from oracle import cnn
    exe, d = driver
    inputs = 1 if x.ndim == 4 else x.shape[1]
    dims = cnn.Dims(x.shape[0], x.shape[-3], x.shape[-2], x.shape[-1], 1 if periodic else 0, 1,
                    inputs, 0, alpha)
    src, dst = str(d / "in.bin"), str(d / "out.bin")
    with open(src, "wb") as f:
        f.write(bytes(oracle.make_cfg(p)))
        f.write(np.int32(nsteps).tobytes())
        for k in FIELDS:
            f.write(np.ascontiguousarray(st[k], dtype=np.float64).tobytes())
        f.write(bytes(dims))
        for a in (params, x, target):
            f.write(np.ascontiguousarray(a, dtype=np.float64).tobytes())
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([exe, src, dst], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "Sanitizer" not in r.stderr, r.stderr[-4000:]
    raw = np.fromfile(dst, dtype=np.uint8)
    n = p["nx"] * p["ny"] * p["nz"]
    off = 0
    out = {}
    for k in FIELDS:
        out[k] = raw[off: off + 8 * n].view(np.float64).reshape(p["nz"], p["ny"], p["nx"])
        off += 8 * n
    nrec = nsteps * p["n_subiter"]
    rb = C.sizeof(oracle.OSolve) * nrec
    recs = (oracle.OSolve * nrec).from_buffer_copy(raw[off: off + rb].tobytes())
    off += rb
    diag = raw[off: off + 8 * (6 + 9 * p["nz"])].view(np.float64)
    off += 8 * (6 + 9 * p["nz"])
    m = target.size
    y = raw[off: off + 8 * m].view(np.float64).reshape(target.shape)
    off += 8 * m
    loss = float(raw[off: off + 8].view(np.float64)[0])
    off += 8
    grad = raw[off:].view(np.float64)
    return out, [(r.sweeps, r.status, r.guess) for r in recs], diag, y, loss, grad


CASES = [
    (dict(name="C1m", nx=10, ny=7, nz=16, poisson_tol=1e-9, poisson_scheme="chebyshev",
          guess="previous", mean_mode="exact"), 1, False, (2, 10, 12, 13)),
    (dict(name="C1i", nx=9, ny=6, poisson_tol=1e-9, poisson_scheme="jacobi",
          guess="extrapolate", mean_mode="level", advection="weno3", wall="free_slip"),
     3, True, (1, 3, 6, 9, 8)),
]


@pytest.mark.parametrize("case,inputs,periodic,xshape", CASES)
def test_sanitized_oracle_equals_ordinary_build(driver, case, inputs, periodic, xshape):
    import oracle
    from oracle import cnn
    kw = dict(case)
    p = li.workload(kw.pop("name"), **kw)
    st0 = li.initial_state(p)
    rng = np.random.default_rng(3)
    for k in ("u", "v", "w"):
        st0[k] = st0[k] + 0.3 * rng.standard_normal(st0[k].shape)
    params = 0.2 * rng.standard_normal(cnn.param_count(inputs))
    x = rng.standard_normal(xshape)
    ys, xs = cnn.layer_size(xshape[-2], xshape[-1], cnn.LAYERS, periodic)
    target = rng.standard_normal((xshape[0], xshape[-3], ys, xs))

    got, grecs, diag, y, loss, grad = _run(driver, p, st0, 2, params, x, target, periodic)

    ref = {k: v.copy() for k, v in st0.items()}
    recs, _ = oracle.step(p, ref, nsteps=2)
    assert grecs == [(r["sweeps"], r["status"], r["guess"]) for r in recs]
    for k in FIELDS:
        assert np.array_equal(got[k], ref[k]), k
    d = oracle.diagnostics(p, ref)
    want = [d[k] for k in ("mass_thl", "mass_qt", "div_l2", "div_max", "cfl", "ke")]
    assert np.array_equal(diag[:6], np.array(want))
    prof = np.stack([d["profiles"][k] for k in ("thl", "qt", "ql", "u", "v", "w", "w2", "w3", "b")])
    assert np.array_equal(diag[6:].reshape(9, p["nz"]), prof)
    out, acts, pre = cnn.forward(params, x, periodic=periodic)
    l_ref, gy = cnn.loss(out, target, p["dx"], p["dy"], p["dz"])
    g_ref = cnn.backward(params, x, acts, pre, gy, periodic=periodic)
    assert np.array_equal(y, out)
    assert loss == l_ref
    assert np.array_equal(grad, g_ref)


@pytest.mark.parametrize("body,report", [
    ("double *a = malloc(4 * sizeof(double)); a[0] = argc; free(a); printf(\"%f\\n\", a[argc]);",
     "heap-use-after-free"),
    ("int k = 2147483600 + argc * 100; printf(\"%d\\n\", k);", "runtime error"),
])
def test_sanitizer_build_reports_planted_errors(driver, body, report):
    """The same flags catch a use after free (AddressSanitizer) and a signed
    overflow (UndefinedBehaviorSanitizer), so a clean run of the oracle
    above means something."""
    _, d = driver
    src, exe = str(d / "planted.c"), str(d / "planted")
    with open(src, "w") as f:
        f.write("#include <stdio.h>\n#include <stdlib.h>\n"
                "int main(int argc, char **argv) { (void)argv; " + body + " return 0; }\n")
    r = subprocess.run(["gcc", *FLAGS, src, "-o", exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([exe], capture_output=True, text=True, timeout=60,
                       env=dict(os.environ, UBSAN_OPTIONS="halt_on_error=1"))
    assert r.returncode != 0 and report in r.stderr, (r.returncode, r.stderr[-2000:])
