"""ctypes access to the 2D oracle stepper (oracle/stepper2d.c).

TEST INFRASTRUCTURE: see oracle/__init__.py.
"""
from __future__ import annotations

import ctypes as C
import os
import threading
from typing import Dict, Optional

import numpy as np

from . import build as _build

_P_D = C.POINTER(C.c_double)
_P_I64 = C.POINTER(C.c_int64)


class _Problem(C.Structure):
    _fields_ = [
        ("pol", C.c_int32), ("abc", C.c_int32),
        ("nx", C.c_int64), ("nz", C.c_int64),
        ("S", C.c_double), ("beta", C.c_double),
        ("eps_rest", _P_D), ("mu_rest", _P_D),
        ("src_row", C.c_int64), ("src_profile", _P_D),
        ("src_amp", C.c_double), ("src_omega", C.c_double),
        ("src_t0", C.c_double), ("src_tau", C.c_double),
        ("src_phase", C.c_double), ("src_t_off", C.c_double),
        ("nprobe", C.c_int32), ("probe_x", _P_I64), ("probe_z", _P_I64),
        ("nfreq", C.c_int32), ("omegas", _P_D),
        ("init_d", _P_D), ("init_b", _P_D), ("init_c", _P_D),
    ]


class _Result(C.Structure):
    _fields_ = [("trace", _P_D), ("dft_re", _P_D), ("dft_im", _P_D),
                ("final_d", _P_D), ("final_b", _P_D), ("final_c", _P_D)]


_lib = None
_lock = threading.Lock()


def load(path: str):
    """Load a compiled 2D stepper (the oracle's own, or a test's variant)."""
    lib = C.CDLL(path)
    lib.oracle2d_solve.argtypes = [C.POINTER(_Problem), C.c_int64,
                                   C.POINTER(_Result)]
    lib.oracle2d_solve.restype = C.c_int
    return lib


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_build.LIB2D):
                _build.build()
            _lib = load(_build.LIB2D)
    return _lib


def _ptr(a, ctype=_P_D):
    if a is None:
        return C.cast(None, ctype)
    return a.ctypes.data_as(ctype)


def solve(problem, steps: Optional[int] = None, fields: bool = True,
          lib=None) -> Dict[str, np.ndarray]:
    """Run the FP64 2D oracle on a workloads.Problem2D.  Returns 'trace'
    (nprobe, steps), 'dft' (nprobe, nfreq complex) and, if `fields`, the
    final 'd', 'b', 'c' as (nx, nz) arrays (column i, z index k)."""
    lib = _load() if lib is None else lib
    p = problem
    steps = int(p.steps if steps is None else steps)
    nx, nz = int(p.nx), int(p.nz)
    f64 = lambda a: None if a is None else np.ascontiguousarray(a, dtype=np.float64)
    eps, mu = f64(p.eps_rest), f64(p.mu_rest)
    prof = f64(p.src_profile)
    px = np.ascontiguousarray(p.probe_x, dtype=np.int64)
    pz = np.ascontiguousarray(p.probe_z, dtype=np.int64)
    om = f64(p.omegas)
    init = [None if getattr(p, k, None) is None else f64(np.reshape(getattr(p, k), (nx * nz,)))
            for k in ("init_d", "init_b", "init_c")]
    pr = _Problem(int(p.pol), int(p.abc), nx, nz, float(p.courant), float(p.beta),
                  _ptr(eps), _ptr(mu), int(p.src_row), _ptr(prof),
                  float(p.pulse.amp), float(p.pulse.omega), float(p.pulse.t0),
                  float(p.pulse.tau), float(p.pulse.phase), float(p.pulse.t_off),
                  len(px), _ptr(px, _P_I64), _ptr(pz, _P_I64), len(om), _ptr(om),
                  _ptr(init[0]), _ptr(init[1]), _ptr(init[2]))
    trace = np.zeros((len(px), steps))
    dre = np.zeros((len(px), len(om)))
    dim = np.zeros((len(px), len(om)))
    out = {}
    if fields:
        for k in ("d", "b", "c"):
            out[k] = np.zeros((nx, nz))
    res = _Result(_ptr(trace), _ptr(dre), _ptr(dim), _ptr(out.get("d")),
                  _ptr(out.get("b")), _ptr(out.get("c")))
    rc = lib.oracle2d_solve(C.byref(pr), steps, C.byref(res))
    if rc != 0:
        raise ValueError(f"oracle2d_solve rejected the problem (code {rc})")
    out["trace"] = trace
    out["dft"] = dre + 1j * dim
    return out
