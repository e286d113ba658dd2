"""CPU checks of the C ABI: the library loads, exports every function that
include/les.h declares, the ctypes structs match the C layouts, argument
validation fails cleanly, and the workspace layout is consistent.  No GPU
compute calls."""
import ctypes as C
import os
import re
import subprocess

import pytest

import les_inputs as li
from conftest import ROOT, load_table1


def declared_functions():
    names = set()
    for h in ("les.h", "les_cnn.h"):
        src = open(os.path.join(ROOT, "include", h)).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        names |= set(re.findall(r"\b(les_[a-z0-9_]+)\s*\(", src))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    from paper_2301_04698_amd import les
    return les


def test_exports_every_declared_symbol(lib):
    from paper_2301_04698_amd import cnn
    L = lib.load()
    cnn.lib()
    names = declared_functions()
    assert set(names) == set(lib.EXPORTS) | set(cnn.EXPORTS), names
    for n in names:
        assert hasattr(L, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", lib.LIB_PATH], capture_output=True, text=True)
    exported = set(re.findall(r" T (les_\w+)", out.stdout))
    assert set(names) <= exported


def test_struct_layouts_match_header(lib, tmp_path):
    prog = tmp_path / "sz.c"
    prog.write_text(r'''
#include "les.h"
#include <stdio.h>
#include <stddef.h>
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(les_config), sizeof(les_buffers),
         sizeof(les_solve_stats), sizeof(les_poisson_opts), sizeof(les_step_opts),
         sizeof(les_step_stats), sizeof(les_diag), offsetof(les_config, dx),
         offsetof(les_config, satadj_tol), offsetof(les_step_stats, res_rel_max));
  return 0;
}''')
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(prog), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True).stdout.split()]
    want = [C.sizeof(lib.LesConfig), C.sizeof(lib.LesBuffers), C.sizeof(lib.LesSolveStats),
            C.sizeof(lib.LesPoissonOpts), C.sizeof(lib.LesStepOpts), C.sizeof(lib.LesStepStats),
            C.sizeof(lib.LesDiag), lib.LesConfig.dx.offset, lib.LesConfig.satadj_tol.offset,
            lib.LesStepStats.res_rel_max.offset]
    assert got == want


def test_default_config_is_table1(lib):
    c = lib.default_config()
    for k, v in load_table1().items():
        assert getattr(c, k) == v, k


def test_make_config_carries_every_parameter(lib, oracle_lib):
    for guess in ("zero", "extrapolate", "previous"):
        p = li.workload("C2", guess=guess)
        c = lib.make_config(p)
        o = oracle_lib.make_cfg(p)
        for name, _ in oracle_lib.OCfg._fields_:
            if name not in ("reserved", "guess_passes"):
                assert getattr(c, name) == getattr(o, name), name
        assert c.precision == lib.LES_FP32 and c.poisson_scheme == lib.LES_CHEBYSHEV


@pytest.mark.parametrize("override,needle", [
    (dict(nz=3), "4 <= nz <= 65535"),
    (dict(nz=65536, nx=2, ny=1), "4 <= nz <= 65535"),
    (dict(mean_mode=5), "mean mode"),
    (dict(guess="learned", guess_passes=5), "guess_passes"),
    (dict(guess="previous", guess_passes=2), "guess_passes"),
    (dict(guess_passes=-1), "guess_passes"),
    (dict(ny=0), "nx must be >= 2, ny >= 1"),
    (dict(nx=1), "nx must be >= 2, ny >= 1"),
    (dict(wall=7), "wall condition"),
    (dict(nu_const=-1.0), "nu_const"),
    (dict(nx=16384, ny=16385, nz=4), "grid too large"),  # FP64 plane just over 2 GiB
    (dict(nx=32768, ny=32768, nz=4, precision="fp32"), "grid too large"),
    (dict(dt=0.0), "> 0"),
    (dict(poisson_tol=0.0), "poisson_tol"),
    (dict(poisson_check_every=0), "check_every"),
    (dict(n_subiter=0), "n_subiter"),
    (dict(jacobi_omega=2.5), "jacobi_omega"),
])
def test_invalid_config_rejected(lib, override, needle):
    c = lib.make_config(li.workload("C1", **override))
    assert lib.workspace_bytes(c) == 0
    assert needle in lib.last_error()


def test_plane_limit_is_per_precision(lib):
    """The 2 GiB bound on one z plane: a 16384 x 16385 plane is 1 GiB in
    FP32 (accepted; only sized here, nothing is allocated) and just over
    2 GiB in FP64 (rejected)."""
    c = lib.make_config(li.workload("C1", nx=16384, ny=16385, nz=4, precision="fp32"))
    assert lib.workspace_bytes(c) > 25 * 16384 * 16385 * 4 * 4
    c = lib.make_config(li.workload("C1", nx=16384, ny=16385, nz=4, precision="fp64"))
    assert lib.workspace_bytes(c) == 0


def test_init_rejects_null_buffers(lib):
    c = lib.make_config(li.workload("C1"))
    b = lib.LesBuffers()
    h = C.c_void_p()
    rc = lib.load().les_init(C.byref(c), C.byref(b), None, C.byref(h))
    assert rc == lib.LES_ERR_ARG and "NULL" in lib.last_error()
    assert not h.value


def test_init_rejects_small_workspace(lib):
    c = lib.make_config(li.workload("C1"))
    fake = 1 << 40  # never dereferenced: validation fails first
    b = lib.LesBuffers(*([fake] * 7), 16)
    h = C.c_void_p()
    rc = lib.load().les_init(C.byref(c), C.byref(b), None, C.byref(h))
    assert rc == lib.LES_ERR_ARG and "workspace" in lib.last_error()


def test_workspace_layout(lib):
    for name in ("C1", "C2", "C5"):
        p = li.workload(name)
        c = lib.make_config(p)
        total = lib.workspace_bytes(c)
        n = p["nx"] * p["ny"] * p["nz"]
        es = 8 if c.precision == lib.LES_FP64 else 4
        offs = [lib.workspace_offset(c, f) for f in lib.WS_FIELDS]
        assert offs == sorted(offs) and all(o % 256 == 0 for o in offs)
        assert all(b - a >= n * es for a, b in zip(offs, offs[1:]))
        assert offs[-1] + n * es <= total
    c5 = lib.make_config(li.workload("C5"))
    assert lib.workspace_bytes(c5) < 32 * 2 ** 30  # fits easily in 288 GB of HBM


# ------------------------------------------------------ guess network ABI

def test_cnn_dims_layout_and_counts(lib, oracle_lib, tmp_path):
    from oracle import cnn as ocnn
    from paper_2301_04698_amd import cnn
    prog = tmp_path / "cz.c"
    prog.write_text(r'''
#include "les_cnn.h"
#include <stdio.h>
#include <stddef.h>
int main(void) {
  printf("%zu %zu\n", sizeof(les_cnn_dims), offsetof(les_cnn_dims, alpha));
  return 0;
}''')
    exe = tmp_path / "cz"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(prog), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True).stdout.split()]
    assert got == [C.sizeof(cnn.CnnDims), cnn.CnnDims.alpha.offset]
    assert cnn.param_count() == ocnn.param_count() == 14737
    assert cnn.param_count(3) == ocnn.param_count(3) == 15601
    for inputs in (1, 3):
        for l in range(4):
            assert cnn.weight_offset(l, inputs) == ocnn.weight_offset(l, inputs)
            assert cnn.bias_offset(l, inputs) == ocnn.bias_offset(l, inputs)
    with pytest.raises(lib.LesError):
        cnn.param_count(2)


def test_cnn_work_bytes_validation(lib):
    from paper_2301_04698_amd import cnn
    ok = cnn.dims((2, 16, 20, 21), periodic=False)
    assert cnn.work_bytes(ok) > 2 * 16 * 20 * 21 * (2 + 3 * 32)
    three = cnn.dims((2, 3, 16, 20, 21), periodic=False)
    assert three.inputs == 3
    assert cnn.work_bytes(three) - cnn.work_bytes(ok) >= 2 * 16 * 20 * 21 * 2 * 2
    for bad in (cnn.dims((0, 16, 20, 20)), cnn.dims((1, 16, 10, 20)),
                cnn.dims((1, 16, 20, 20), alpha=-1.0), cnn.dims((1, 2, 16, 20, 20))):
        with pytest.raises(lib.LesError):
            cnn.work_bytes(bad)
    assert cnn.work_bytes(cnn.dims((1, 8, 5, 5), periodic=True)) > 0


def test_learned_guess_workspace(lib):
    p = li.workload("C1")
    base = lib.workspace_bytes(lib.make_config(p))
    prev = lib.workspace_bytes(lib.make_config(dict(p, guess="previous")))
    learned = lib.workspace_bytes(lib.make_config(dict(p, guess="learned")))
    n = p["nx"] * p["ny"] * p["nz"]
    assert prev >= base + p["n_subiter"] * n * 8
    # residual, network input, two 16-channel activations and the parameters
    assert learned >= prev + n * (4 + 2 + 2 * 32) + 14737 * 6
    # the three-input form: the previous pressure, the extrapolated base,
    # three input channels and the larger parameter vector
    learned3 = lib.workspace_bytes(lib.make_config(dict(p, guess="learned3")))
    assert learned3 >= base + n * 8 + n * (4 + 6 + 2 * 32) + 15601 * 6
