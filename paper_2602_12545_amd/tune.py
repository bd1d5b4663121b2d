"""Autotuning front end: runs fld_tune / fld_batch_tune (timing on the GPU, in
the library) and keeps the winners in a JSON cache keyed by grid shape and the
options that fix the numerics, so later runs skip the search.

The cache file is plain JSON: {key: {"options": {...}, "threads": n, "ms": t}}.
Its path is the `cache` argument, else $FLD_TUNE_CACHE, else no cache.
"""
from __future__ import annotations

import ctypes
import hashlib
import json
import os
from typing import Optional, Sequence

from ._binding import (FLDError, FLD_OK, _P, _I, _D, _ptr, _stream_handle, default_options, fld_bc, fld_grid,
                       fld_options, fld_tune_entry, lib)

_NUMERIC = ("precision", "limiter", "norm", "rel_tol", "max_inner", "inner_rtol")
_TUNED = ("smoother", "mg_coarse_max", "mg_coarse_op", "chunk", "use_graph", "mg_cycle")


def _opt_dict(o: fld_options) -> dict:
    return {k: getattr(o, k) for k, _ in o._fields_}


def _opt_from(d: dict, base: fld_options) -> fld_options:
    o = fld_options()
    ctypes.memmove(ctypes.byref(o), ctypes.byref(base), ctypes.sizeof(o))
    for k in _TUNED:
        if k in d:
            setattr(o, k, d[k])
    return o


def _cache_path(cache: Optional[str]) -> Optional[str]:
    return cache if cache is not None else os.environ.get("FLD_TUNE_CACHE")


def _load(path):
    if not path or not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


def _store(path, key, value):
    if not path:
        return
    data = _load(path)
    data[key] = value
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _key(kind: str, shape, base: fld_options, extra=()) -> str:
    desc = {"kind": kind, "shape": shape, "numerics": {k: getattr(base, k) for k in _NUMERIC}, "extra": list(extra)}
    return kind + ":" + hashlib.sha1(json.dumps(desc, sort_keys=True).encode()).hexdigest()[:16]


def _table(entries, n):
    return [{"options": {k: getattr(entries[i].opt, k) for k in _TUNED}, "threads": entries[i].threads,
             "status": entries[i].status, "inner_iters": entries[i].inner_iters, "ms": entries[i].ms}
            for i in range(min(n, len(entries)))]


def tune_grid(nx: int, ny: int, geom: int, x_faces, y_faces, bcs: Sequence, fields: dict, dt: float,
              base: Optional[fld_options] = None, reps: int = 2, cache: Optional[str] = None, stream=None):
    """Best options for one grid.  fields: torch float64 GPU tensors E, T, rho,
    kappa_R, kappa_P, c_v (and ghost_E or None).  Returns (options, table);
    table is None when the result came from the cache."""
    import numpy as np
    base = base if base is not None else default_options()
    xf = np.ascontiguousarray(x_faces, dtype=np.float64)
    yf = np.ascontiguousarray(y_faces, dtype=np.float64)
    kinds = [int(b[0] if isinstance(b, tuple) else b.kind) for b in bcs]
    key = _key("grid", [nx, ny, geom], base,
               [hashlib.sha1(xf.tobytes() + yf.tobytes()).hexdigest()[:12], kinds])
    path = _cache_path(cache)
    hit = _load(path).get(key)
    if hit is not None:
        return _opt_from(hit["options"], base), None
    g = fld_grid()
    g.nx, g.ny, g.geom = nx, ny, geom
    g.x_faces = xf.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    g.y_faces = yf.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    for s, b in enumerate(bcs):
        kind, value = (b if isinstance(b, tuple) else (b.kind, b.value))
        g.bc[s].kind, g.bc[s].value = int(kind), float(value)
    best = fld_options()
    entries = (fld_tune_entry * 256)()  # the whole candidate table (132 entries)
    n = _I()
    f = fields
    st = lib.fld_tune(ctypes.byref(g), ctypes.byref(base), _ptr(f["E"]), _ptr(f["T"]), _ptr(f["rho"]),
                      _ptr(f["kappa_R"]), _ptr(f["kappa_P"]), _ptr(f["c_v"]), _ptr(f.get("ghost_E")), float(dt),
                      int(reps), ctypes.byref(best), entries, len(entries), ctypes.byref(n), _stream_handle(stream))
    if st != FLD_OK:
        raise FLDError(st, "no candidate configuration converged" if st == 4 else "fld_tune")
    table = _table(entries, n.value)
    best_ms = min(e["ms"] for e in table if e["status"] == 0)
    _store(path, key, {"options": {k: getattr(best, k) for k in _TUNED}, "threads": 0, "ms": best_ms})
    return best, table


def tune_batch(nx: Sequence[int], ny: Sequence[int], dx: Sequence[float], dy: Sequence[float], fields: dict,
               dt: float, bcs: Optional[Sequence] = None, base: Optional[fld_options] = None, reps: int = 2,
               cache: Optional[str] = None, stream=None):
    """Best (options, threads) for a batch of blocks; fields are packed.
    Returns (options, threads, table); table is None on a cache hit."""
    base = base if base is not None else default_options()
    nb = len(nx)
    key = _key("batch", [list(map(int, nx)), list(map(int, ny))], base,
               [list(map(float, dx)), list(map(float, dy))])
    path = _cache_path(cache)
    hit = _load(path).get(key)
    if hit is not None:
        return _opt_from(hit["options"], base), int(hit["threads"]), None
    anx, any_ = (_I * nb)(*map(int, nx)), (_I * nb)(*map(int, ny))
    adx, ady = (_D * nb)(*map(float, dx)), (_D * nb)(*map(float, dy))
    bc_arr = None
    if bcs is not None:
        bc_arr = (fld_bc * 4)()
        for s, b in enumerate(bcs):
            kind, value = (b if isinstance(b, tuple) else (b.kind, b.value))
            bc_arr[s].kind, bc_arr[s].value = int(kind), float(value)
    best = fld_options()
    threads = _I()
    entries = (fld_tune_entry * 16)()
    n = _I()
    f = fields
    st = lib.fld_batch_tune(nb, anx, any_, adx, ady, bc_arr, ctypes.byref(base), _ptr(f["E"]), _ptr(f["T"]),
                            _ptr(f["rho"]), _ptr(f["kappa_R"]), _ptr(f["kappa_P"]), _ptr(f["c_v"]),
                            _ptr(f.get("ghost_E")), float(dt), int(reps), ctypes.byref(best),
                            ctypes.byref(threads), entries, 16, ctypes.byref(n), _stream_handle(stream))
    if st != FLD_OK:
        raise FLDError(st, "no candidate configuration converged" if st == 4 else "fld_batch_tune")
    table = _table(entries, n.value)
    best_ms = min(e["ms"] for e in table if e["status"] == 0)
    _store(path, key, {"options": {k: getattr(best, k) for k in _TUNED}, "threads": threads.value, "ms": best_ms})
    return best, threads.value, table
