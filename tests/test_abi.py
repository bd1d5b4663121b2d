"""The C-ABI library loads on the CPU and exports every entry point that
include/fld.h declares; the ctypes structures match the C layout."""
import ctypes
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fld.h")
LIB = os.path.join(ROOT, "paper_2602_12545_amd", "libfld.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*(fld_[a-z_0-9]+)\s*\(", src, flags=re.M)
    return sorted(set(names))


needs_lib = pytest.mark.skipif(not os.path.exists(LIB), reason="libfld.so not built")


def test_header_declares_the_boundary():
    names = declared_functions()
    for f in ("fld_create", "fld_assemble", "fld_solve", "fld_step", "fld_steps", "fld_substep", "fld_face_flux", "fld_set_mass_flux", "fld_set_cv_law", "fld_gas_update",
              "fld_get_operator", "fld_destroy", "fld_default_options", "fld_batch_create", "fld_batch_step",
              "fld_batch_steps", "fld_batch_destroy"):
        assert f in names


@needs_lib
def test_every_declared_symbol_is_exported():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    for n in declared_functions():
        assert re.search(rf"\bT {n}\b", out), n


@needs_lib
def test_host_only_entry_points_run_without_gpu():
    lib = ctypes.CDLL(LIB)
    lib.fld_version.restype = ctypes.c_char_p
    assert lib.fld_version().startswith(b"fld-mi355x")
    lib.fld_status_string.restype = ctypes.c_char_p
    assert lib.fld_status_string(4) == b"tolerance not reached"
    lib.fld_create.restype = ctypes.c_int32
    assert lib.fld_create(None, None, None, None) == 1  # EINVAL before any device call
    lib.fld_set_mass_flux.restype = ctypes.c_int32
    assert lib.fld_set_mass_flux(None, None, None) == 1
    lib.fld_set_cv_law.restype = ctypes.c_int32
    lib.fld_set_cv_law.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_double]
    assert lib.fld_set_cv_law(None, 1.0, 1.5) == 1
    lib.fld_substep.restype = ctypes.c_int32
    n_done = ctypes.c_int32(7)
    assert lib.fld_substep(None, None, None, None, None, None, None, None, ctypes.c_double(1.0), 1,
                           ctypes.c_double(1.5), ctypes.c_double(0.0), 1, None, None, ctypes.byref(n_done), None,
                           None) == 1
    lib.fld_face_flux.restype = ctypes.c_int32
    assert lib.fld_face_flux(None, None, None, None, ctypes.c_double(1.0), 0) == 1
    lib.fld_batch_last_error.restype = ctypes.c_char_p
    out = ctypes.c_void_p()
    assert lib.fld_batch_create(ctypes.byref(out), 0, None, None, None, None, None, None, None) == 1
    assert out.value is None
    assert b"nblocks" in lib.fld_batch_last_error(None)


def c_layout():
    code = r'''
#include <stdio.h>
#include <stddef.h>
#include "fld.h"
int main(void) {
  printf("%zu %zu %zu %zu\n", sizeof(fld_bc), sizeof(fld_grid), sizeof(fld_options), sizeof(fld_solve_info));
  printf("%zu %zu %zu %zu\n", offsetof(fld_grid, bc), offsetof(fld_options, rel_tol),
         offsetof(fld_options, inner_rtol), offsetof(fld_solve_info, rel_resid));
  printf("%zu %zu %zu\n", offsetof(fld_options, use_graph), offsetof(fld_solve_info, ms),
         offsetof(fld_options, mg_cycle));
  return 0;
}
'''
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "l.c")
        exe = os.path.join(d, "l")
        open(src, "w").write(code)
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), src, "-o", exe], check=True)
        return [int(v) for v in subprocess.run([exe], capture_output=True, text=True).stdout.split()]


@needs_lib
def test_ctypes_structures_match_c_layout():
    from paper_2602_12545_amd import _binding as B
    c = c_layout()
    py = [ctypes.sizeof(B.fld_bc), ctypes.sizeof(B.fld_grid), ctypes.sizeof(B.fld_options),
          ctypes.sizeof(B.fld_solve_info), B.fld_grid.bc.offset, B.fld_options.rel_tol.offset,
          B.fld_options.inner_rtol.offset, B.fld_solve_info.rel_resid.offset, B.fld_options.use_graph.offset,
          B.fld_solve_info.ms.offset, B.fld_options.mg_cycle.offset]
    assert c == py


@needs_lib
def test_noalloc_block_step_rejects_before_touching_the_device():
    """fld_block_step_noalloc checks sizes and arguments on the host first:
    a bad side, and a block whose workspace exceeds the static 4 MiB, are
    refused with EINVAL and a reason, without any GPU call."""
    import paper_2602_12545_amd._binding as B  # noqa: F401  (ctypes signatures)
    lib = B.lib
    opt = B.default_options(precision=B.FLD_FP64)
    dummy = ctypes.c_void_p(16)
    args = lambda nx, ny: (nx, ny, 1e10, 1e10, None, ctypes.byref(opt), dummy, dummy, dummy, dummy, dummy, dummy,
                           dummy, 1e4, None, None)
    assert lib.fld_block_step_noalloc(*args(0, 8)) == B.FLD_EINVAL
    assert b"block sides" in lib.fld_batch_last_error(None)
    assert lib.fld_block_step_noalloc(*args(512, 512)) == B.FLD_EINVAL
    assert b"bytes of workspace" in lib.fld_batch_last_error(None)
    opt.precision = B.FLD_MIXED
    assert lib.fld_block_step_noalloc(*args(256, 256)) == B.FLD_EINVAL


@needs_lib
def test_forest_validation_runs_on_the_host():
    """fld_forest_create refuses overlapping, unbalanced and non-covering
    forests, and non-FP64 options, before touching the device."""
    import paper_2602_12545_amd._binding as B
    lib = B.lib
    opt = B.default_options(precision=B.FLD_FP64)

    def create(blocks, nx0=8, ny0=8, o=opt):
        arr = (B.fld_forest_block * len(blocks))(*[B.fld_forest_block(*b) for b in blocks])
        h = ctypes.c_void_p()
        return lib.fld_forest_create(ctypes.byref(h), len(blocks), arr, nx0, ny0, 1e10, 1e10, None, ctypes.byref(o),
                                     None)

    assert create([(0, 0, 0, 4, 4), (0, 2, 2, 4, 4)]) == B.FLD_EINVAL
    assert b"overlaps" in lib.fld_forest_last_error(None)
    assert create([(0, 0, 0, 8, 4)]) == B.FLD_EINVAL
    assert b"cover" in lib.fld_forest_last_error(None)
    assert create([(0, 0, 0, 4, 8), (2, 16, 0, 16, 32)]) == B.FLD_EINVAL
    assert b"balanced" in lib.fld_forest_last_error(None)
    assert create([(0, 0, 0, 8, 8), (1, 0, 0, 2, 2)]) == B.FLD_EINVAL
    mixed = B.default_options(precision=B.FLD_MIXED)
    assert create([(0, 0, 0, 8, 8)], o=mixed) == B.FLD_EINVAL
