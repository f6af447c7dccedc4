"""C-ABI checks that need no GPU: exported symbols, struct layouts shared by
include/fvib.h and the ctypes binding, and the descriptor validation that
runs before any device work."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fvib.h")


def _abi():
    from paper_2505_23940_amd import _abi
    return _abi


def _lib():
    return _abi().load()


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fvib_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = _lib()
    names = declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) <= set(_abi().EXPORTS), set(names) - set(_abi().EXPORTS)


def test_struct_layouts_match_header(tmp_path):
    """Compile a probe against the header with the host compiler and compare
    sizes and offsets with the ctypes mirror."""
    A = _abi()
    probe = tmp_path / "probe.c"
    probe.write_text(r'''
#include <stddef.h>
#include <stdio.h>
#include "fvib.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu\n", sizeof(fvib_grid_desc), sizeof(fvib_body_desc),
         sizeof(fvib_fields), sizeof(fvib_adjoint), sizeof(fvib_step_info));
  printf("%zu %zu %zu %zu %zu %zu\n", offsetof(fvib_grid_desc, bc_vel), offsetof(fvib_grid_desc, nu),
         offsetof(fvib_grid_desc, poisson_tol), offsetof(fvib_grid_desc, inner_rtol),
         offsetof(fvib_grid_desc, check_every), offsetof(fvib_grid_desc, solver));
  printf("%zu %zu %zu\n", offsetof(fvib_body_desc, free_dof), offsetof(fvib_body_desc, m),
         offsetof(fvib_step_info, force));
  return 0;
}
''')
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-I", os.path.dirname(HEADER), str(probe), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    sizes = [int(x) for x in out[0].split()]
    offs = [int(x) for x in out[1].split()]
    offs2 = [int(x) for x in out[2].split()]
    assert sizes == [C.sizeof(A.GridDesc), C.sizeof(A.BodyDesc), C.sizeof(A.Fields),
                     C.sizeof(A.Adjoint), C.sizeof(A.StepInfo)]
    assert offs == [A.GridDesc.bc_vel.offset, A.GridDesc.nu.offset, A.GridDesc.poisson_tol.offset,
                    A.GridDesc.inner_rtol.offset, A.GridDesc.check_every.offset,
                    A.GridDesc.solver.offset]
    assert offs2 == [A.BodyDesc.free_dof.offset, A.BodyDesc.m.offset, A.StepInfo.force.offset]


def _desc(**over):
    A = _abi()
    d = A.GridDesc()
    d.dim = 2
    d.n[0], d.n[1], d.n[2] = 8, 6, 1
    fx = np.linspace(0.0, 1.0, 9)
    fy = np.linspace(0.0, 1.0, 7)
    keep = [fx, fy]
    d.faces[0] = fx.ctypes.data
    d.faces[1] = fy.ctypes.data
    for a in range(3):
        d.bc[a][0] = d.bc[a][1] = A.BC["periodic"]
    d.nu, d.rho, d.dt, d.u_conv = 0.01, 1.0, 1e-3, 1.0
    d.convection, d.precision, d.solver = 0, 0, 1
    d.poisson_tol, d.poisson_maxit, d.ir_maxit, d.inner_rtol, d.check_every = 1e-10, 100, 10, 1e-4, 8
    for k, v in over.items():
        if k == "faces_y":
            keep.append(v)
            d.faces[1] = v.ctypes.data
        elif k == "bc":
            for (a, s), val in v.items():
                d.bc[a][s] = val
        else:
            setattr(d, k, v)
    return d, keep


@pytest.mark.parametrize("case,over", [
    ("dim", {"dim": 4}),
    ("unpaired periodic", {"bc": {(0, 0): 0, (0, 1): 1}}),
    ("unknown bc", {"bc": {(1, 0): 9, (1, 1): 9}}),
    ("decreasing faces", {"faces_y": np.array([0.0, 0.3, 0.2, 0.5, 0.7, 0.9, 1.0])}),
    ("non-uniform periodic", {"faces_y": np.array([0.0, 0.1, 0.3, 0.5, 0.7, 0.9, 1.0])}),
    ("nu", {"nu": 0.0}),
    ("dt", {"dt": -1.0}),
    ("tol", {"poisson_tol": 0.0}),
    ("maxit", {"poisson_maxit": 0}),
    ("solver", {"solver": 7}),
    ("precision", {"precision": 5}),
    ("ir", {"ir_maxit": 0}),
])
def test_create_rejects_invalid_descriptors(case, over):
    A = _abi()
    lib = _lib()
    d, keep = _desc(**over)
    h = C.c_void_p(123)
    rc = lib.fvib_create_grid(C.byref(d), None, C.byref(h))
    assert rc == A.FVIB_EINVAL, (case, rc)
    assert h.value is None
    assert lib.fvib_last_error(None).decode() != ""


def test_null_arguments_are_rejected():
    A = _abi()
    lib = _lib()
    assert lib.fvib_create_grid(None, None, None) == A.FVIB_EINVAL
    assert lib.fvib_destroy_grid(None) == A.FVIB_EINVAL
    assert lib.fvib_step(None, None, None, None) == A.FVIB_EINVAL
    assert lib.fvib_step_adjoint(None, None, None, None, None, None) == A.FVIB_EINVAL
    shape = (C.c_int64 * 3)()
    strides = (C.c_int64 * 3)()
    assert lib.fvib_field_layout(None, 0, shape, strides, None) == A.FVIB_EINVAL
    assert lib.fvib_timing_enable(None, 1) == A.FVIB_EINVAL
    assert lib.fvib_version().decode().startswith("fvib")


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    A = _abi()
    monkeypatch.setattr(A, "_LIB", None)
    with pytest.raises(RuntimeError):
        A.load(str(tmp_path / "missing.so"))
