"""ctypes access to the C oracle stepper (oracle/stepper.c).

TEST INFRASTRUCTURE: see oracle/__init__.py.
"""
from __future__ import annotations

import ctypes as C
import os
import threading
from concurrent.futures import ThreadPoolExecutor
from typing import Dict, List, Optional, Sequence

import numpy as np

from . import build as _build

_P_D = C.POINTER(C.c_double)
_P_I64 = C.POINTER(C.c_int64)


class _Problem(C.Structure):
    _fields_ = [
        ("nz", C.c_int64), ("S", C.c_double), ("beta", C.c_double),
        ("kind", C.c_int32), ("abc", C.c_int32),
        ("eps_rest", _P_D), ("mu_rest", _P_D),
        ("src_cell", C.c_int64),
        ("src_amp", C.c_double), ("src_omega", C.c_double),
        ("src_t0", C.c_double), ("src_tau", C.c_double),
        ("src_phase", C.c_double), ("src_t_off", C.c_double),
        ("nprobe", C.c_int32), ("probe_cells", _P_I64),
        ("nfreq", C.c_int32), ("omegas", _P_D),
        ("init_d", _P_D), ("init_b", _P_D),
        ("windowed", C.c_int32), ("t_on", C.c_double), ("t_off", C.c_double),
        ("eps_bg", C.c_double), ("mu_bg", C.c_double),
    ]


class _Result(C.Structure):
    _fields_ = [("trace", _P_D), ("dft_re", _P_D), ("dft_im", _P_D),
                ("final_d", _P_D), ("final_b", _P_D),
                ("final_es", _P_D), ("final_hs", _P_D)]


_lib = None
_lock = threading.Lock()


def load(path: str):
    """A stepper library at `path` (the oracle's own, or a test's variant
    compiled by build.compile_stepper), ready for solve(..., lib=...)."""
    lib = C.CDLL(path)
    lib.oracle_solve.argtypes = [C.POINTER(_Problem), C.c_int64,
                                 C.POINTER(_Result)]
    lib.oracle_solve.restype = C.c_int
    return lib


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_build.LIB):
                _build.build()
            _lib = load(_build.LIB)
    return _lib


def _ptr(a: Optional[np.ndarray], ctype=_P_D):
    if a is None:
        return C.cast(None, ctype)
    return a.ctypes.data_as(ctype)


def solve(problem, steps: Optional[int] = None,
          init_d: Optional[np.ndarray] = None,
          init_b: Optional[np.ndarray] = None,
          fields: bool = True, lib=None) -> Dict[str, np.ndarray]:
    """Run the FP64 oracle on a workloads.Problem.

    Returns a dict with 'trace' (nprobe, steps), 'dft' (nprobe, nfreq,
    complex), and, if `fields`, 'd', 'b', 'es', 'hs' (nz each) at the end.
    The initial fields default to the problem's init_d / init_b (zero when
    absent).
    """
    lib = _load() if lib is None else lib
    p = problem
    if init_d is None:
        init_d = getattr(p, "init_d", None)
    if init_b is None:
        init_b = getattr(p, "init_b", None)
    steps = int(p.steps if steps is None else steps)
    nz = int(p.nz)
    eps = np.ascontiguousarray(p.eps_rest, dtype=np.float64)
    mu = np.ascontiguousarray(p.mu_rest, dtype=np.float64)
    probes = np.ascontiguousarray(p.probes, dtype=np.int64)
    omegas = np.ascontiguousarray(p.omegas, dtype=np.float64)
    if init_d is not None:
        init_d = np.ascontiguousarray(init_d, dtype=np.float64)
        assert init_d.shape == (nz,)
    if init_b is not None:
        init_b = np.ascontiguousarray(init_b, dtype=np.float64)
        assert init_b.shape == (nz,)
    pr = _Problem(nz, float(p.courant), float(p.beta), int(p.kind), int(p.abc),
                  _ptr(eps), _ptr(mu), int(p.src_cell),
                  float(p.pulse.amp), float(p.pulse.omega), float(p.pulse.t0),
                  float(p.pulse.tau), float(p.pulse.phase), float(p.pulse.t_off),
                  len(probes), _ptr(probes, _P_I64), len(omegas), _ptr(omegas),
                  _ptr(init_d), _ptr(init_b))
    win = getattr(p, "window", None)
    if win is not None:
        pr.windowed = 1
        pr.t_on, pr.t_off = float(win.t_on), float(win.t_off)
        pr.eps_bg, pr.mu_bg = float(win.eps_bg), float(win.mu_bg)
    nprobe, nfreq = len(probes), len(omegas)
    trace = np.zeros((nprobe, steps))
    dre = np.zeros((nprobe, nfreq))
    dim = np.zeros((nprobe, nfreq))
    out = {}
    if fields:
        for key in ("d", "b", "es", "hs"):
            out[key] = np.zeros(nz)
    res = _Result(_ptr(trace), _ptr(dre), _ptr(dim),
                  _ptr(out.get("d")), _ptr(out.get("b")),
                  _ptr(out.get("es")), _ptr(out.get("hs")))
    rc = lib.oracle_solve(C.byref(pr), steps, C.byref(res))
    if rc != 0:
        raise ValueError(f"oracle_solve rejected the problem (code {rc})")
    out["trace"] = trace
    out["dft"] = dre + 1j * dim
    return out


def solve_many(problems: Sequence, threads: int, fields: bool = False
               ) -> List[Dict[str, np.ndarray]]:
    """Independent oracle runs over a thread pool (the C call releases the
    interpreter lock, so runs proceed in parallel, one per thread)."""
    with ThreadPoolExecutor(max_workers=max(1, threads)) as ex:
        return list(ex.map(lambda q: solve(q, fields=fields), problems))
