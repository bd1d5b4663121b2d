"""ctypes binding of libfld (include/fld.h).

Argument marshalling only: torch tensors are passed as device pointers, the
current HIP stream as the context stream.  Every computation runs in the HIP
kernels of libfld.so; if the library is missing the import fails loudly.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfld.so")

FLD_OK, FLD_EINVAL, FLD_ENOMEM, FLD_EHIP, FLD_ENOCONV, FLD_EBREAKDOWN, FLD_ENONFINITE, FLD_ENOTREADY = range(8)
FLD_CARTESIAN, FLD_SPHERICAL_POLAR = 0, 1
(FLD_BC_REFLECT, FLD_BC_DIRICHLET_FACE, FLD_BC_DIRICHLET_GHOST, FLD_BC_FLUX_IN, FLD_BC_FREE_STREAM,
 FLD_BC_AXIS) = range(6)
FLD_FP64, FLD_FP32, FLD_MIXED = 0, 1, 2
FLD_LIMITER_LP, FLD_LIMITER_MINERBO, FLD_LIMITER_DIFFUSION = 0, 1, 2
FLD_NORM_ROW, FLD_NORM_SCALED = 0, 1
FLD_MG_GALERKIN, FLD_MG_HALVED = 0, 1
FLD_SMOOTH_LINE, FLD_SMOOTH_POINT, FLD_SMOOTH_LINE_SPLIT = 0, 1, 2
FLD_MG_CYCLE_V, FLD_MG_CYCLE_K, FLD_MG_CYCLE_W2, FLD_MG_CYCLE_KL_K, FLD_MG_CYCLE_KL_W2 = range(5)

PRECISIONS = {"fp64": FLD_FP64, "fp32": FLD_FP32, "mixed": FLD_MIXED}


class fld_bc(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("value", ctypes.c_double)]


class fld_grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("geom", ctypes.c_int32),
                ("x_faces", ctypes.POINTER(ctypes.c_double)), ("y_faces", ctypes.POINTER(ctypes.c_double)),
                ("bc", fld_bc * 4)]


class fld_options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("limiter", ctypes.c_int32), ("norm", ctypes.c_int32),
                ("rel_tol", ctypes.c_double), ("max_outer", ctypes.c_int32), ("max_inner", ctypes.c_int32),
                ("inner_rtol", ctypes.c_double), ("mg_coarse_max", ctypes.c_int32),
                ("mg_coarse_op", ctypes.c_int32), ("smoother", ctypes.c_int32), ("chunk", ctypes.c_int32),
                ("use_graph", ctypes.c_int32), ("mg_cycle", ctypes.c_int32)]


class fld_solve_info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("outer_iters", ctypes.c_int32), ("inner_iters", ctypes.c_int32),
                ("mg_levels", ctypes.c_int32), ("rel_resid", ctypes.c_double), ("rel_resid_row", ctypes.c_double),
                ("rel_resid_scaled", ctypes.c_double), ("ms", ctypes.c_float)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class fld_forest_block(ctypes.Structure):
    _fields_ = [("level", ctypes.c_int32), ("i0", ctypes.c_int32), ("j0", ctypes.c_int32), ("nx", ctypes.c_int32),
                ("ny", ctypes.c_int32)]


class fld_tune_entry(ctypes.Structure):
    _fields_ = [("opt", fld_options), ("threads", ctypes.c_int32), ("status", ctypes.c_int32),
                ("inner_iters", ctypes.c_int32), ("ms", ctypes.c_float)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libfld.so not built ({LIB_PATH}); run __graft_entry__.build() or "
                          "python paper_2602_12545_amd/build.py")
    # torch bundles its own HIP runtime under the same soname as the system
    # one libfld.so links against; whichever loads first serves the process.
    # Loading torch first keeps torch's kernels on the runtime they were built
    # for (the other order makes its launches fail as invalid device functions).
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    return ctypes.CDLL(LIB_PATH)


lib = _load()

_P = ctypes.c_void_p
_D = ctypes.c_double
_I = ctypes.c_int32
_SIGS = {
    "fld_default_options": (None, [ctypes.POINTER(fld_options)]),
    "fld_create": (_I, [ctypes.POINTER(_P), ctypes.POINTER(fld_grid), ctypes.POINTER(fld_options), _P]),
    "fld_assemble": (_I, [_P, _P, _P, _P, _P, _P, _P, _P, _D]),
    "fld_solve": (_I, [_P, _P, ctypes.POINTER(fld_solve_info)]),
    "fld_gas_update": (_I, [_P, _P, _P]),
    "fld_step": (_I, [_P, _P, _P, _P, _P, _P, _P, _P, _D, ctypes.POINTER(fld_solve_info)]),
    "fld_steps": (_I, [_P, _I, _P, _P, _P, _P, _P, _P, _P, _D, ctypes.POINTER(fld_solve_info)]),
    "fld_steps_graph": (_I, [_P, _I, _P, _P, _P, _P, _P, _P, _P, _D, ctypes.POINTER(fld_solve_info)]),
    "fld_substep": (_I, [_P, _P, _P, _P, _P, _P, _P, _P, _D, _I, _D, _D, _I, ctypes.POINTER(_D),
                         ctypes.POINTER(fld_solve_info), ctypes.POINTER(_I), _P, _P]),
    "fld_face_flux": (_I, [_P, _P, _P, _P, _D, _I]),
    "fld_set_mass_flux": (_I, [_P, _P, _P]),
    "fld_set_cv_law": (_I, [_P, ctypes.c_double, ctypes.c_double]),
    "fld_get_operator": (_I, [_P, _P, _P, _P, _P]),
    "fld_mg_levels": (_I, [_P]),
    "fld_profile": (_I, [_P, _I]),
    "fld_profile_overhead": (_I, [_P, _I, ctypes.POINTER(ctypes.c_double)]),
    "fld_profile_sweeps": (_I, [_P, _I, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_I)]),
    "fld_profile_sweeps_levels": (_I, [_P, _I, _I, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_I)]),
    "fld_profile_sweeps_range": (_I, [_P, _I, _I, _I, ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(_I)]),
    "fld_profile_read": (_I, [_P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double),
                              ctypes.POINTER(ctypes.c_double)]),
    "fld_status_string": (ctypes.c_char_p, [_I]),
    "fld_last_error": (ctypes.c_char_p, [_P]),
    "fld_version": (ctypes.c_char_p, []),
    "fld_destroy": (None, [_P]),
    "fld_batch_create": (_I, [ctypes.POINTER(_P), _I, ctypes.POINTER(_I), ctypes.POINTER(_I),
                              ctypes.POINTER(_D), ctypes.POINTER(_D), ctypes.POINTER(fld_bc),
                              ctypes.POINTER(fld_options), _P]),
    "fld_batch_step": (_I, [_P, _P, _P, _P, _P, _P, _P, _P, _D, ctypes.POINTER(fld_solve_info)]),
    "fld_batch_steps": (_I, [_P, _I, _P, _P, _P, _P, _P, _P, _P, _D, ctypes.POINTER(fld_solve_info)]),
    "fld_batch_set_threads": (_I, [_P, _I]),
    "fld_batch_get_threads": (_I, [_P, ctypes.POINTER(_I)]),
    "fld_batch_sizes": (_I, [_P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]),
    "fld_batch_last_error": (ctypes.c_char_p, [_P]),
    "fld_batch_destroy": (None, [_P]),
    "fld_block_step_noalloc": (_I, [_I, _I, _D, _D, ctypes.POINTER(fld_bc), ctypes.POINTER(fld_options), _P, _P, _P,
                                    _P, _P, _P, _P, _D, _P, ctypes.POINTER(fld_solve_info)]),
    "fld_forest_create": (_I, [ctypes.POINTER(_P), _I, ctypes.POINTER(fld_forest_block), _I, _I, _D, _D,
                               ctypes.POINTER(fld_bc), ctypes.POINTER(fld_options), _P]),
    "fld_forest_sizes": (_I, [_P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                              ctypes.POINTER(ctypes.c_int64)]),
    "fld_forest_cells": (_I, [_P, ctypes.POINTER(_D), ctypes.POINTER(_D), ctypes.POINTER(_I)]),
    "fld_forest_step": (_I, [_P, _P, _P, _P, _P, _P, _P, _D, ctypes.POINTER(fld_solve_info)]),
    "fld_forest_last_error": (ctypes.c_char_p, [_P]),
    "fld_forest_destroy": (None, [_P]),
    "fld_tune": (_I, [ctypes.POINTER(fld_grid), ctypes.POINTER(fld_options), _P, _P, _P, _P, _P, _P, _P, _D, _I,
                      ctypes.POINTER(fld_options), ctypes.POINTER(fld_tune_entry), _I, ctypes.POINTER(_I), _P]),
    "fld_batch_tune": (_I, [_I, ctypes.POINTER(_I), ctypes.POINTER(_I), ctypes.POINTER(_D), ctypes.POINTER(_D),
                            ctypes.POINTER(fld_bc), ctypes.POINTER(fld_options), _P, _P, _P, _P, _P, _P, _P, _D, _I,
                            ctypes.POINTER(fld_options), ctypes.POINTER(_I), ctypes.POINTER(fld_tune_entry), _I,
                            ctypes.POINTER(_I), _P]),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(lib, _name)
    _f.restype = _res
    _f.argtypes = _args


class FLDError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{lib.fld_status_string(status).decode()} ({status}): {msg}")
        self.status = status


def default_options(**kw) -> fld_options:
    o = fld_options()
    lib.fld_default_options(ctypes.byref(o))
    for k, v in kw.items():
        if k == "precision" and isinstance(v, str):
            v = PRECISIONS[v]
        setattr(o, k, v)
    return o


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch tensor")
    if not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError("fields must be contiguous float64 tensors on the GPU")
    return t.data_ptr()


def _stream_handle(stream) -> Optional[int]:
    if stream is not None:
        return int(stream)
    import torch
    return torch.cuda.current_stream().cuda_stream or None


class Context:
    """One grid: wraps fld_create ... fld_destroy.  Fields are torch float64 GPU tensors [ny, nx]."""

    def __init__(self, nx: int, ny: int, geom: int, x_faces, y_faces, bcs: Sequence, options=None, stream=None):
        import numpy as np
        self._xf = np.ascontiguousarray(x_faces, dtype=np.float64)
        self._yf = np.ascontiguousarray(y_faces, dtype=np.float64)
        if self._xf.size != nx + 1 or self._yf.size != ny + 1:
            raise ValueError("face arrays must have nx+1 and ny+1 entries")
        g = fld_grid()
        g.nx, g.ny, g.geom = nx, ny, geom
        g.x_faces = self._xf.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        g.y_faces = self._yf.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        for s, b in enumerate(bcs):
            kind, value = (b if isinstance(b, tuple) else (b.kind, b.value))
            g.bc[s].kind, g.bc[s].value = int(kind), float(value)
        self.options = options if options is not None else default_options()
        self.nx, self.ny = nx, ny
        h = _P()
        st = lib.fld_create(ctypes.byref(h), ctypes.byref(g), ctypes.byref(self.options), _stream_handle(stream))
        if st != FLD_OK:
            msg = lib.fld_last_error(h).decode() if h.value else ""
            lib.fld_destroy(h)
            raise FLDError(st, msg)
        self.handle = h

    def _check(self, st):
        if st != FLD_OK:
            raise FLDError(st, lib.fld_last_error(self.handle).decode())

    def assemble(self, E, T, rho, kappa_R, kappa_P, c_v, dt, ghost_E=None):
        self._check(lib.fld_assemble(self.handle, _ptr(E), _ptr(T), _ptr(rho), _ptr(kappa_R), _ptr(kappa_P),
                                     _ptr(c_v), _ptr(ghost_E), float(dt)))

    def solve(self, E, check=True) -> dict:
        info = fld_solve_info()
        st = lib.fld_solve(self.handle, _ptr(E), ctypes.byref(info))
        if check:
            self._check(st)
        return info.as_dict()

    def gas_update(self, E, T_out):
        self._check(lib.fld_gas_update(self.handle, _ptr(E), _ptr(T_out)))

    def step(self, E, T, rho, kappa_R, kappa_P, c_v, dt, ghost_E=None, check=True) -> dict:
        info = fld_solve_info()
        st = lib.fld_step(self.handle, _ptr(E), _ptr(T), _ptr(rho), _ptr(kappa_R), _ptr(kappa_P), _ptr(c_v),
                          _ptr(ghost_E), float(dt), ctypes.byref(info))
        if check:
            self._check(st)
        return info.as_dict()

    def steps(self, nsteps, E, T, rho, kappa_R, kappa_P, c_v, dt, ghost_E=None, check=True):
        infos = (fld_solve_info * max(1, nsteps))()
        st = lib.fld_steps(self.handle, int(nsteps), _ptr(E), _ptr(T), _ptr(rho), _ptr(kappa_R), _ptr(kappa_P),
                           _ptr(c_v), _ptr(ghost_E), float(dt), infos)
        if check:
            self._check(st)
        return [infos[k].as_dict() for k in range(nsteps)]

    def steps_graph(self, nsteps, E, T, rho, kappa_R, kappa_P, c_v, dt, ghost_E=None, check=True):
        """fld_steps_graph: the steps after the first replay one captured step
        graph (the context then serves only further steps_graph calls)."""
        infos = (fld_solve_info * max(1, nsteps))()
        st = lib.fld_steps_graph(self.handle, int(nsteps), _ptr(E), _ptr(T), _ptr(rho), _ptr(kappa_R),
                                 _ptr(kappa_P), _ptr(c_v), _ptr(ghost_E), float(dt), infos)
        if check:
            self._check(st)
        return [infos[k].as_dict() for k in range(nsteps)]

    def substep(self, E, T, rho, kappa_R, kappa_P, c_v, dt, ghost_E=None, n_sub=1, q=1.0, dbar=0.0,
                max_sub=10000, check=True, Fx=None, Fy=None):
        """One step of length dt as sub-steps: the geometric series (n_sub, q)
        when dbar == 0, else coupling-limited with factor dbar; Fx, Fy (device
        tensors, optional) receive the sub-step-averaged face fluxes.  Returns
        {"status", "dts", "infos"} (one entry per sub-step taken)."""
        cap = max(1, int(max_sub))
        dts = (ctypes.c_double * cap)()
        infos = (fld_solve_info * cap)()
        n = _I()
        st = lib.fld_substep(self.handle, _ptr(E), _ptr(T), _ptr(rho), _ptr(kappa_R), _ptr(kappa_P), _ptr(c_v),
                             _ptr(ghost_E), float(dt), int(n_sub), float(q), float(dbar), int(max_sub), dts, infos,
                             ctypes.byref(n), _ptr(Fx), _ptr(Fy))
        if check:
            self._check(st)
        return {"status": st, "dts": [dts[k] for k in range(n.value)],
                "infos": [infos[k].as_dict() for k in range(n.value)]}

    def face_flux(self, E, Fx=None, Fy=None, w=1.0, accumulate=False):
        """Face fluxes of the last assembled step from E into Fx [ny][nx+1],
        Fy [ny+1][nx] (device tensors), scaled by w, added if accumulate."""
        self._check(lib.fld_face_flux(self.handle, _ptr(E), _ptr(Fx), _ptr(Fy), float(w), 1 if accumulate else 0))

    def set_mass_flux(self, fx=None, fy=None):
        """Face mass fluxes of the explicit advection term (device tensors
        [ny][nx+1] and [ny+1][nx], or None); kept referenced while set."""
        self._check(lib.fld_set_mass_flux(self.handle, _ptr(fx), _ptr(fy)))
        self._mass_flux = (fx, fy)

    def set_cv_law(self, T_ref: float = 1.0, p: float = 0.0):
        """Power-law heat capacity c_v(T) = c_v (T / T_ref)^p, re-evaluated
        from T before every later step's assembly (p = 0: off)."""
        self._check(lib.fld_set_cv_law(self.handle, float(T_ref), float(p)))

    def get_operator(self):
        import torch
        shape = (self.ny, self.nx)
        out = [torch.empty(shape, dtype=torch.float64, device="cuda") for _ in range(4)]
        self._check(lib.fld_get_operator(self.handle, *[_ptr(t) for t in out]))
        return dict(zip(("W_e", "W_n", "diag", "rhs"), out))

    def profile(self, enable: bool = True):
        self._check(lib.fld_profile(self.handle, 1 if enable else 0))

    def profile_read(self) -> dict:
        n = ctypes.c_int64()
        ms = ctypes.c_double()
        by = ctypes.c_double()
        self._check(lib.fld_profile_read(self.handle, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(by)))
        return {"launches": n.value, "ms": ms.value, "bytes": by.value}

    def profile_overhead(self, reps: int = 200) -> float:
        us = ctypes.c_double()
        self._check(lib.fld_profile_overhead(self.handle, int(reps), ctypes.byref(us)))
        return us.value

    def profile_sweeps(self, reps: int = 50, levels: int = 0, first: int = 0) -> dict:
        us, fl, by, n = ctypes.c_double(), ctypes.c_double(), ctypes.c_double(), _I()
        self._check(lib.fld_profile_sweeps_range(self.handle, int(first), int(levels), int(reps), ctypes.byref(us),
                                                 ctypes.byref(fl), ctypes.byref(by), ctypes.byref(n)))
        return {"us_per_launch": us.value, "floor_us": fl.value, "bytes_per_launch": by.value, "launches": n.value}

    @property
    def mg_levels(self) -> int:
        return lib.fld_mg_levels(self.handle)

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            lib.fld_destroy(self.handle)
            self.handle = _P()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Independent Cartesian blocks solved together: wraps fld_batch_create ...
    fld_batch_destroy.  Fields are packed torch float64 GPU tensors (block after
    block, each row-major [ny, nx])."""

    def __init__(self, nx: Sequence[int], ny: Sequence[int], dx: Sequence[float], dy: Sequence[float],
                 bcs: Optional[Sequence] = None, options=None, stream=None):
        nb = len(nx)
        if not (len(ny) == len(dx) == len(dy) == nb):
            raise ValueError("nx, ny, dx, dy must have one entry per block")
        anx, any_ = (_I * nb)(*[int(v) for v in nx]), (_I * nb)(*[int(v) for v in ny])
        adx, ady = (_D * nb)(*[float(v) for v in dx]), (_D * nb)(*[float(v) for v in dy])
        bc_arr = None
        if bcs is not None:
            bc_arr = (fld_bc * 4)()
            for s, b in enumerate(bcs):
                kind, value = (b if isinstance(b, tuple) else (b.kind, b.value))
                bc_arr[s].kind, bc_arr[s].value = int(kind), float(value)
        self.options = options if options is not None else default_options()
        self.nblocks = nb
        h = _P()
        st = lib.fld_batch_create(ctypes.byref(h), nb, anx, any_, adx, ady, bc_arr, ctypes.byref(self.options),
                                  _stream_handle(stream))
        if st != FLD_OK:
            raise FLDError(st, lib.fld_batch_last_error(None).decode())
        self.handle = h
        cells, ghosts = ctypes.c_int64(), ctypes.c_int64()
        lib.fld_batch_sizes(h, ctypes.byref(cells), ctypes.byref(ghosts))
        self.cells, self.ghosts = cells.value, ghosts.value

    def _check(self, st):
        if st != FLD_OK:
            raise FLDError(st, lib.fld_batch_last_error(self.handle).decode())

    def step(self, E, T, rho, kappa_R, kappa_P, c_v, dt, ghost_E=None, check=True, records=True):
        infos = (fld_solve_info * self.nblocks)() if records else None
        st = lib.fld_batch_step(self.handle, _ptr(E), _ptr(T), _ptr(rho), _ptr(kappa_R), _ptr(kappa_P), _ptr(c_v),
                                _ptr(ghost_E), float(dt), infos)
        if check:
            self._check(st)
        return [infos[k].as_dict() for k in range(self.nblocks)] if records else None

    def steps(self, nsteps, E, T, rho, kappa_R, kappa_P, c_v, dt, ghost_E=None, check=True):
        infos = (fld_solve_info * self.nblocks)()
        st = lib.fld_batch_steps(self.handle, int(nsteps), _ptr(E), _ptr(T), _ptr(rho), _ptr(kappa_R),
                                 _ptr(kappa_P), _ptr(c_v), _ptr(ghost_E), float(dt), infos)
        if check:
            self._check(st)
        return [infos[k].as_dict() for k in range(self.nblocks)]

    @property
    def threads(self) -> int:
        v = _I()
        self._check(lib.fld_batch_get_threads(self.handle, ctypes.byref(v)))
        return v.value

    @threads.setter
    def threads(self, n: int):
        self._check(lib.fld_batch_set_threads(self.handle, int(n)))

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            lib.fld_batch_destroy(self.handle)
            self.handle = _P()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Forest:
    """A statically refined block forest solved as one matrix: wraps
    fld_forest_create ... fld_forest_destroy.  blocks: (level, i0, j0, nx, ny)
    tuples; fields are torch float64 GPU tensors of `cells` values in cell
    order (block after block, each row-major)."""

    def __init__(self, blocks, nx0: int, ny0: int, dx0: float, dy0: float, bcs: Optional[Sequence] = None,
                 options=None, stream=None):
        nb = len(blocks)
        arr = (fld_forest_block * nb)(*[fld_forest_block(*[int(v) for v in b]) for b in blocks])
        bc_arr = None
        if bcs is not None:
            bc_arr = (fld_bc * 4)()
            for s, b in enumerate(bcs):
                kind, value = (b if isinstance(b, tuple) else (b.kind, b.value))
                bc_arr[s].kind, bc_arr[s].value = int(kind), float(value)
        self.options = options if options is not None else default_options(precision="fp64")
        h = _P()
        st = lib.fld_forest_create(ctypes.byref(h), nb, arr, int(nx0), int(ny0), float(dx0), float(dy0), bc_arr,
                                   ctypes.byref(self.options), _stream_handle(stream))
        if st != FLD_OK:
            raise FLDError(st, lib.fld_forest_last_error(None).decode())
        self.handle = h
        c, f, b = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        lib.fld_forest_sizes(h, ctypes.byref(c), ctypes.byref(f), ctypes.byref(b))
        self.cells, self.faces, self.boundary_faces = c.value, f.value, b.value

    def centres(self):
        import numpy as np
        x = (_D * self.cells)()
        y = (_D * self.cells)()
        lv = (_I * self.cells)()
        lib.fld_forest_cells(self.handle, x, y, lv)
        return np.ctypeslib.as_array(x).copy(), np.ctypeslib.as_array(y).copy(), np.ctypeslib.as_array(lv).copy()

    def step(self, E, T, rho, kappa_R, kappa_P, c_v, dt, check=True) -> dict:
        info = fld_solve_info()
        st = lib.fld_forest_step(self.handle, _ptr(E), _ptr(T), _ptr(rho), _ptr(kappa_R), _ptr(kappa_P),
                                 _ptr(c_v), float(dt), ctypes.byref(info))
        if check and st != FLD_OK:
            raise FLDError(st, lib.fld_forest_last_error(self.handle).decode())
        out = info.as_dict()
        out["call_status"] = st
        return out

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            lib.fld_forest_destroy(self.handle)
            self.handle = _P()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def block_step_noalloc(nx: int, ny: int, dx: float, dy: float, E, T, rho, kappa_R, kappa_P, c_v, dt, ghost_E=None,
                       bcs: Optional[Sequence] = None, options=None, stream=None, check=True) -> dict:
    """One block stepped as one block of a batch, with the library's static
    per-device workspace (fld_block_step_noalloc: no device allocation)."""
    bc_arr = None
    if bcs is not None:
        bc_arr = (fld_bc * 4)()
        for s, b in enumerate(bcs):
            kind, value = (b if isinstance(b, tuple) else (b.kind, b.value))
            bc_arr[s].kind, bc_arr[s].value = int(kind), float(value)
    opt = options if options is not None else default_options()
    info = fld_solve_info()
    st = lib.fld_block_step_noalloc(int(nx), int(ny), float(dx), float(dy), bc_arr, ctypes.byref(opt), _ptr(E),
                                    _ptr(T), _ptr(rho), _ptr(kappa_R), _ptr(kappa_P), _ptr(c_v), _ptr(ghost_E),
                                    float(dt), _stream_handle(stream), ctypes.byref(info))
    if check and st != FLD_OK:
        raise FLDError(st, lib.fld_batch_last_error(None).decode())
    out = info.as_dict()
    out["call_status"] = st
    return out
