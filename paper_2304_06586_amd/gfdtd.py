"""Python binding of the generalized-FDTD C-ABI (include/gfdtd.h).

Argument marshalling only: every step of the solve runs in the HIP
kernels of libgfdtd.so.  PyTorch provides device memory (workspaces and
server pools are torch uint8 tensors) and the stream.  There is no CPU
path: if the native library is missing the calls raise.

Problem descriptors are duck-typed: any object with the attributes of
`workloads.Problem` (nz, steps, courant, beta, kind, precision, abc,
flags, eps_rest, mu_rest, src_cell, pulse.{amp, omega, t0, tau, phase,
t_off}, probes, omegas, and optionally init_d / init_b and window
(t_on, t_off, eps_bg, mu_bg)); 2D ones those of `workloads.Problem2D`.
"""
from __future__ import annotations

import ctypes as C
import os
import threading
from typing import Dict, List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgfdtd.so")

GFDTD_OK = 0
GFDTD_E_INVALID = 1
GFDTD_E_UNSTABLE = 2
GFDTD_E_NOMEM = 3
GFDTD_E_DEVICE = 4
GFDTD_E_NOT_READY = 5
GFDTD_E_BLOWUP = 6
GFDTD_E_UNSUPPORTED = 7

GFDTD_MODULATION = 0
GFDTD_MATTER = 1
GFDTD_F32 = 0
GFDTD_F64 = 1
GFDTD_ABC_MUR1 = 0
GFDTD_ABC_PEC = 1
GFDTD_ABC_PERIODIC = 2
GFDTD_FLAG_RECORD_TRACE = 1
GFDTD_FLAG_ALLOW_UNSTABLE = 2
GFDTD_FLAG_KEEP_FIELDS = 4
GFDTD_FLAG_TIME_WINDOW = 8
GFDTD_STATIC_WORKSPACE_BYTES = 32 << 20
GFDTD_VARIANT_AUTO = 0
GFDTD_VARIANT_STEP = 1
GFDTD_VARIANT_TILED = 2

_PD = C.POINTER(C.c_double)
_PI64 = C.POINTER(C.c_int64)


class gfdtd_problem(C.Structure):
    _fields_ = [
        ("struct_size", C.c_uint32), ("kind", C.c_int32),
        ("precision", C.c_int32), ("abc", C.c_int32), ("flags", C.c_uint32),
        ("nprobe", C.c_int32), ("nfreq", C.c_int32), ("reserved0", C.c_int32),
        ("nz", C.c_int64), ("courant", C.c_double), ("beta", C.c_double),
        ("eps_rest", _PD), ("mu_rest", _PD), ("src_cell", C.c_int64),
        ("src_amp", C.c_double), ("src_omega", C.c_double),
        ("src_t0", C.c_double), ("src_tau", C.c_double),
        ("src_phase", C.c_double), ("src_t_off", C.c_double),
        ("probe_cells", _PI64), ("omegas", _PD),
        ("init_d", _PD), ("init_b", _PD),
        ("t_on", C.c_double), ("t_off", C.c_double),
        ("eps_bg", C.c_double), ("mu_bg", C.c_double),
    ]


class gfdtd_result(C.Structure):
    _fields_ = [
        ("struct_size", C.c_uint32), ("run_status", C.c_int32),
        ("steps_done", C.c_int64), ("trace", _PD), ("dft_re", _PD),
        ("dft_im", _PD), ("final_d", _PD), ("final_b", _PD),
    ]


class gfdtd_exec(C.Structure):
    _fields_ = [
        ("struct_size", C.c_uint32), ("variant", C.c_int32),
        ("cells_per_lane", C.c_int32), ("block_steps", C.c_int32),
        ("use_graph", C.c_int32), ("tile_waves", C.c_int32),
        ("exchange_steps", C.c_int32), ("reserved0", C.c_int32),
    ]


class gfdtd_stats(C.Structure):
    _fields_ = [
        ("struct_size", C.c_uint32), ("cells_per_lane", C.c_int32),
        ("block_steps", C.c_int32), ("graph", C.c_int32),
        ("launches", C.c_int64), ("tiles", C.c_int64),
        ("cell_updates", C.c_double), ("step_ms", C.c_double),
        ("pass_ms", C.c_double), ("tile_waves", C.c_int32),
        ("exchange_steps", C.c_int32), ("streams", C.c_int32),
        ("reserved", C.c_int32),
    ]


class gfdtd_server_config(C.Structure):
    _fields_ = [
        ("struct_size", C.c_uint32), ("max_slots", C.c_int32),
        ("block_steps", C.c_int32), ("max_ahead", C.c_int32),
        ("pool", C.c_void_p), ("pool_bytes", C.c_size_t),
        ("stream", C.c_void_p),
    ]


GFDTD2D_TE = 0
GFDTD2D_TM = 1


class gfdtd2d_problem(C.Structure):
    _fields_ = [
        ("struct_size", C.c_uint32), ("pol", C.c_int32),
        ("precision", C.c_int32), ("abc", C.c_int32), ("flags", C.c_uint32),
        ("nprobe", C.c_int32), ("nfreq", C.c_int32), ("reserved0", C.c_int32),
        ("nx", C.c_int64), ("nz", C.c_int64),
        ("courant", C.c_double), ("beta", C.c_double),
        ("eps_rest", _PD), ("mu_rest", _PD), ("src_row", C.c_int64),
        ("src_profile", _PD),
        ("src_amp", C.c_double), ("src_omega", C.c_double),
        ("src_t0", C.c_double), ("src_tau", C.c_double),
        ("src_phase", C.c_double), ("src_t_off", C.c_double),
        ("probe_x", _PI64), ("probe_z", _PI64), ("omegas", _PD),
        ("init_d", _PD), ("init_b", _PD), ("init_c", _PD),
    ]


class gfdtd2d_result(C.Structure):
    _fields_ = [
        ("struct_size", C.c_uint32), ("run_status", C.c_int32),
        ("steps_done", C.c_int64), ("trace", _PD), ("dft_re", _PD),
        ("dft_im", _PD), ("final_d", _PD), ("final_b", _PD), ("final_c", _PD),
    ]


class gfdtd2d_exec(C.Structure):
    _fields_ = [
        ("struct_size", C.c_uint32), ("cells_per_lane", C.c_int32),
        ("columns_per_wave", C.c_int32), ("block_steps", C.c_int32),
    ]


class gfdtd2d_stats(C.Structure):
    _fields_ = [
        ("struct_size", C.c_uint32), ("cells_per_lane", C.c_int32),
        ("columns_per_wave", C.c_int32), ("waves", C.c_int32),
        ("launches", C.c_int64), ("cell_updates", C.c_double),
        ("step_ms", C.c_double), ("pass_ms", C.c_double),
        ("block_steps", C.c_int32), ("reserved0", C.c_int32),
    ]


class GfdtdError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"gfdtd status {status}: {message}")
        self.status = status
        self.message = message


_lib = None
_lock = threading.Lock()

class gfdtd_tmm_stack(C.Structure):
    _fields_ = [
        ("struct_size", C.c_uint32), ("nlayers", C.c_int32), ("beta", C.c_double),
        ("eps", _PD), ("mu", _PD), ("widths", _PD),
    ]


EXPORTS = {
    # name: (restype, argtypes)
    "gfdtd_status_str": (C.c_char_p, [C.c_int]),
    "gfdtd_last_error": (C.c_char_p, []),
    "gfdtd_check": (C.c_int, [C.POINTER(gfdtd_problem), C.POINTER(C.c_double)]),
    "gfdtd_result_sizes": (C.c_int, [C.POINTER(gfdtd_problem), C.c_int64,
                                     C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]),
    "gfdtd_workspace_bytes": (C.c_int, [C.POINTER(gfdtd_problem), C.c_int64,
                                        C.POINTER(C.c_size_t)]),
    "gfdtd_batch_workspace_bytes": (C.c_int, [C.POINTER(gfdtd_problem), _PI64,
                                              C.c_int32, C.POINTER(C.c_size_t)]),
    "gfdtd_solve": (C.c_int, [C.POINTER(gfdtd_problem), C.c_int64, C.c_void_p,
                              C.c_size_t, C.c_void_p, C.POINTER(gfdtd_result)]),
    "gfdtd_solve_static": (C.c_int, [C.POINTER(gfdtd_problem), C.c_int64, C.c_void_p,
                                     C.POINTER(gfdtd_result)]),
    "gfdtd_solve_batch": (C.c_int, [C.POINTER(gfdtd_problem), _PI64, C.c_int32,
                                    C.c_void_p, C.c_size_t, C.c_void_p,
                                    C.POINTER(gfdtd_result)]),
    "gfdtd_batch_prepare": (C.c_int, [C.POINTER(gfdtd_problem), _PI64, C.c_int32,
                                      C.POINTER(gfdtd_exec), C.c_void_p, C.c_size_t,
                                      C.c_void_p, C.POINTER(C.c_void_p)]),
    "gfdtd_batch_run": (C.c_int, [C.c_void_p]),
    "gfdtd_batch_collect": (C.c_int, [C.c_void_p, C.POINTER(gfdtd_result)]),
    "gfdtd_batch_stats": (C.c_int, [C.c_void_p, C.POINTER(gfdtd_stats)]),
    "gfdtd_batch_autotune": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(gfdtd_exec)]),
    "gfdtd_batch_destroy": (None, [C.c_void_p]),
    "gfdtd_server_create": (C.c_int, [C.POINTER(gfdtd_server_config),
                                      C.POINTER(C.c_void_p)]),
    "gfdtd_server_submit": (C.c_int, [C.c_void_p, C.POINTER(gfdtd_problem),
                                      C.c_int64, C.POINTER(C.c_uint64)]),
    "gfdtd_server_progress": (C.c_int, [C.c_void_p, C.c_int32,
                                        C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "gfdtd_server_poll": (C.c_int, [C.c_void_p, C.c_uint64, C.POINTER(gfdtd_result)]),
    "gfdtd_server_destroy": (None, [C.c_void_p]),
    "gfdtd_tmm_workspace_bytes": (C.c_int, [C.POINTER(gfdtd_tmm_stack), C.c_int32,
                                            C.c_int32, C.POINTER(C.c_size_t)]),
    "gfdtd_tmm": (C.c_int, [C.POINTER(gfdtd_tmm_stack), C.c_int32, _PD, C.c_int32,
                            C.c_void_p, C.c_size_t, C.c_void_p, _PD, _PD]),
    "gfdtd_tmm_kernel_ms": (C.c_int, [C.POINTER(C.c_double)]),
    # 2D path (include/gfdtd2d.h)
    "gfdtd2d_check": (C.c_int, [C.POINTER(gfdtd2d_problem), C.c_int64,
                                C.POINTER(C.c_double)]),
    "gfdtd2d_workspace_bytes": (C.c_int, [C.POINTER(gfdtd2d_problem), C.c_int64,
                                          C.POINTER(C.c_size_t)]),
    "gfdtd2d_prepare": (C.c_int, [C.POINTER(gfdtd2d_problem), C.c_int64,
                                  C.POINTER(gfdtd2d_exec), C.c_void_p, C.c_size_t,
                                  C.c_void_p, C.POINTER(C.c_void_p)]),
    "gfdtd2d_run_pass": (C.c_int, [C.c_void_p]),
    "gfdtd2d_collect": (C.c_int, [C.c_void_p, C.POINTER(gfdtd2d_result)]),
    "gfdtd2d_get_stats": (C.c_int, [C.c_void_p, C.POINTER(gfdtd2d_stats)]),
    "gfdtd2d_destroy": (None, [C.c_void_p]),
    "gfdtd2d_solve": (C.c_int, [C.POINTER(gfdtd2d_problem), C.c_int64, C.c_void_p,
                                C.c_size_t, C.c_void_p, C.POINTER(gfdtd2d_result)]),
}


def load_library(path: str = LIB_PATH):
    """Load libgfdtd.so (built in-tree by __graft_entry__.build()).  Raises
    if it is missing: there is no fallback path."""
    global _lib
    with _lock:
        if _lib is None:
            # torch first: its HIP runtime (soname libamdhip64.so.7) then
            # satisfies the library's dependency, so the process holds one
            # runtime, the one that owns the torch-allocated device memory
            import torch  # noqa: F401
            if not os.path.exists(path):
                raise RuntimeError(
                    f"{path} is missing: build the HIP library first "
                    "(python -c 'import __graft_entry__ as g; g.build()')")
            lib = C.CDLL(path)
            for name, (res, args) in EXPORTS.items():
                fn = getattr(lib, name)
                fn.restype = res
                fn.argtypes = args
            _lib = lib
    return _lib


def _check(status: int):
    if status != GFDTD_OK:
        lib = load_library()
        raise GfdtdError(status, lib.gfdtd_last_error().decode())


# ---------------------------------------------------------------- marshalling

class _Marshalled:
    """A gfdtd_problem struct plus the numpy arrays it points into."""

    def __init__(self, p, steps: Optional[int] = None):
        self.eps = np.ascontiguousarray(p.eps_rest, dtype=np.float64)
        self.mu = np.ascontiguousarray(p.mu_rest, dtype=np.float64)
        self.probes = np.ascontiguousarray(p.probes, dtype=np.int64)
        self.omegas = np.ascontiguousarray(p.omegas, dtype=np.float64)
        self.steps = int(p.steps if steps is None else steps)
        self.nz = int(p.nz)
        self.nprobe = len(self.probes)
        self.nfreq = len(self.omegas)
        self.precision = int(p.precision)
        s = gfdtd_problem()
        s.struct_size = C.sizeof(gfdtd_problem)
        s.kind = int(p.kind)
        s.precision = int(p.precision)
        s.abc = int(p.abc)
        s.flags = int(p.flags)
        win = getattr(p, "window", None)
        if win is not None:
            s.flags |= GFDTD_FLAG_TIME_WINDOW
            s.t_on, s.t_off = float(win.t_on), float(win.t_off)
            s.eps_bg, s.mu_bg = float(win.eps_bg), float(win.mu_bg)
        s.nprobe = self.nprobe
        s.nfreq = self.nfreq
        s.nz = self.nz
        s.courant = float(p.courant)
        s.beta = float(p.beta)
        s.eps_rest = self.eps.ctypes.data_as(_PD)
        s.mu_rest = self.mu.ctypes.data_as(_PD)
        s.src_cell = int(p.src_cell)
        s.src_amp = float(p.pulse.amp)
        s.src_omega = float(p.pulse.omega)
        s.src_t0 = float(p.pulse.t0)
        s.src_tau = float(p.pulse.tau)
        s.src_phase = float(p.pulse.phase)
        s.src_t_off = float(p.pulse.t_off)
        s.probe_cells = self.probes.ctypes.data_as(_PI64) if self.nprobe else None
        s.omegas = self.omegas.ctypes.data_as(_PD) if self.nfreq else None
        self.init = []
        for name in ("init_d", "init_b"):
            a = getattr(p, name, None)
            if a is not None:
                a = np.ascontiguousarray(a, dtype=np.float64)
                if a.shape != (self.nz,):
                    raise ValueError(f"{name} must hold nz = {self.nz} values")
                self.init.append(a)
                setattr(s, name, a.ctypes.data_as(_PD))
            else:
                setattr(s, name, None)
        self.struct = s


class _ResultBuffers:
    """Host buffers for one gfdtd_result."""

    def __init__(self, m: _Marshalled, fields: bool = True, trace: bool = True):
        self.trace = np.zeros((m.nprobe, m.steps if trace else 0))
        self.dre = np.zeros((m.nprobe, m.nfreq))
        self.dim = np.zeros((m.nprobe, m.nfreq))
        self.d = np.zeros(m.nz) if fields else None
        self.b = np.zeros(m.nz) if fields else None
        r = gfdtd_result()
        r.struct_size = C.sizeof(gfdtd_result)
        r.trace = self.trace.ctypes.data_as(_PD) if self.trace.size else None
        r.dft_re = self.dre.ctypes.data_as(_PD) if self.dre.size else None
        r.dft_im = self.dim.ctypes.data_as(_PD) if self.dim.size else None
        r.final_d = self.d.ctypes.data_as(_PD) if fields else None
        r.final_b = self.b.ctypes.data_as(_PD) if fields else None
        self.struct = r

    def as_dict(self) -> Dict[str, np.ndarray]:
        out = {"trace": self.trace, "dft": self.dre + 1j * self.dim,
               "status": int(self.struct.run_status),
               "steps_done": int(self.struct.steps_done)}
        if self.d is not None:
            out["d"] = self.d
            out["b"] = self.b
        return out


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(int(stream.cuda_stream))


def _device_buffer(nbytes: int):
    import torch
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device="cuda")


def _exec_struct(variant=GFDTD_VARIANT_AUTO, cells_per_lane=0, block_steps=0,
                 use_graph=-1, tile_waves=0, exchange_steps=0):
    e = gfdtd_exec()
    e.struct_size = C.sizeof(gfdtd_exec)
    e.variant = int(variant)
    e.cells_per_lane = int(cells_per_lane)
    e.block_steps = int(block_steps)
    e.use_graph = int(use_graph)
    e.tile_waves = int(tile_waves)
    e.exchange_steps = int(exchange_steps)
    return e


# ------------------------------------------------------------- entry points

def gfdtd_status_str(status: int) -> str:
    return load_library().gfdtd_status_str(int(status)).decode()


def gfdtd_check(problem) -> float:
    """Validate and pre-flight one problem; returns max |zeta|."""
    lib = load_library()
    m = _Marshalled(problem)
    g = C.c_double(0.0)
    _check(lib.gfdtd_check(C.byref(m.struct), C.byref(g)))
    return g.value


def gfdtd_result_sizes(problem, steps: Optional[int] = None):
    lib = load_library()
    m = _Marshalled(problem, steps)
    a, b = C.c_size_t(0), C.c_size_t(0)
    _check(lib.gfdtd_result_sizes(C.byref(m.struct), m.steps, C.byref(a), C.byref(b)))
    return a.value, b.value


def gfdtd_workspace_bytes(problem, steps: Optional[int] = None) -> int:
    lib = load_library()
    m = _Marshalled(problem, steps)
    n = C.c_size_t(0)
    _check(lib.gfdtd_workspace_bytes(C.byref(m.struct), m.steps, C.byref(n)))
    return n.value


def _arrays(problems, steps):
    ms = [_Marshalled(p, None if steps is None else steps[i])
          for i, p in enumerate(problems)]
    arr = (gfdtd_problem * max(1, len(ms)))(*[m.struct for m in ms])
    st = np.array([m.steps for m in ms] or [0], dtype=np.int64)
    return ms, arr, st


def gfdtd_batch_workspace_bytes(problems: Sequence, steps=None) -> int:
    lib = load_library()
    ms, arr, st = _arrays(problems, steps)
    n = C.c_size_t(0)
    _check(lib.gfdtd_batch_workspace_bytes(arr, st.ctypes.data_as(_PI64), len(ms),
                                           C.byref(n)))
    return n.value


def gfdtd_solve(problem, steps: Optional[int] = None, stream=None,
                fields: bool = True) -> Dict[str, np.ndarray]:
    """Plain single solve (synchronous).  Returns trace (nprobe, steps),
    dft (nprobe, nfreq) complex, and the final d, b (FP64 copies)."""
    lib = load_library()
    m = _Marshalled(problem, steps)
    m.struct.flags |= GFDTD_FLAG_RECORD_TRACE
    n = C.c_size_t(0)
    _check(lib.gfdtd_workspace_bytes(C.byref(m.struct), m.steps, C.byref(n)))
    ws = _device_buffer(n.value)
    out = _ResultBuffers(m, fields)
    _check(lib.gfdtd_solve(C.byref(m.struct), m.steps, C.c_void_p(ws.data_ptr()),
                           n.value, _stream_handle(stream), C.byref(out.struct)))
    return out.as_dict()


def gfdtd_solve_static(problem, steps: Optional[int] = None, stream=None,
                       fields: bool = True) -> Dict[str, np.ndarray]:
    """gfdtd_solve without a caller workspace: the library's fixed device
    array (GFDTD_STATIC_WORKSPACE_BYTES per GPU) serves as the workspace and
    no device memory is allocated.  Same results as gfdtd_solve."""
    lib = load_library()
    m = _Marshalled(problem, steps)
    m.struct.flags |= GFDTD_FLAG_RECORD_TRACE
    out = _ResultBuffers(m, fields)
    _check(lib.gfdtd_solve_static(C.byref(m.struct), m.steps, _stream_handle(stream),
                                  C.byref(out.struct)))
    return out.as_dict()


def gfdtd_solve_batch(problems: Sequence, steps=None, stream=None,
                      fields: bool = True) -> List[Dict[str, np.ndarray]]:
    lib = load_library()
    ms, arr, st = _arrays(problems, steps)
    for i in range(len(ms)):
        arr[i].flags |= GFDTD_FLAG_RECORD_TRACE
    n = C.c_size_t(0)
    _check(lib.gfdtd_batch_workspace_bytes(arr, st.ctypes.data_as(_PI64), len(ms),
                                           C.byref(n)))
    ws = _device_buffer(n.value)
    outs = [_ResultBuffers(m, fields) for m in ms]
    res = (gfdtd_result * max(1, len(ms)))(*[o.struct for o in outs])
    _check(lib.gfdtd_solve_batch(arr, st.ctypes.data_as(_PI64), len(ms),
                                 C.c_void_p(ws.data_ptr()), n.value,
                                 _stream_handle(stream), res))
    for o, r in zip(outs, res):
        o.struct = r
    return [o.as_dict() for o in outs]


def _tmm_stack_dtype():
    """numpy record type laid out as gfdtd_tmm_stack (pointers as uint64)."""
    f = gfdtd_tmm_stack
    names = ["struct_size", "nlayers", "beta", "eps", "mu", "widths"]
    formats = [np.uint32, np.int32, np.float64, np.uint64, np.uint64, np.uint64]
    return np.dtype({"names": names, "formats": formats,
                     "offsets": [getattr(f, k).offset for k in names],
                     "itemsize": C.sizeof(f)})


def _tmm_structs(stacks):
    """The gfdtd_tmm_stack array of `stacks`, filled column-wise: every
    stack's layers are packed into flat arrays (kept alive by the returned
    list) and the records point into them."""
    n = len(stacks)
    eps = [np.ascontiguousarray(st.eps, dtype=np.float64).ravel() for st in stacks]
    widths = [np.ascontiguousarray(st.widths, dtype=np.float64).ravel() for st in stacks]
    mus = [None if st.mu is None else np.ascontiguousarray(st.mu, dtype=np.float64).ravel()
           for st in stacks]
    nl = np.array([len(e) for e in eps], dtype=np.int64)
    nw = np.array([len(w) for w in widths], dtype=np.int64)
    if np.any(nw != np.maximum(nl - 2, 0)):
        raise ValueError("widths must hold the inner layers' widths")
    for e, m in zip(eps, mus):
        if m is not None and m.shape != e.shape:
            raise ValueError("mu must have one value per layer")
    eps_flat = np.concatenate(eps) if n else np.zeros(1)
    w_flat = np.concatenate(widths) if n and nw.sum() else np.zeros(1)
    rec = np.zeros(max(1, n), dtype=_tmm_stack_dtype())
    keep = [eps_flat, w_flat, rec]
    if n:
        rec["struct_size"][:] = C.sizeof(gfdtd_tmm_stack)
        rec["nlayers"][:] = nl
        rec["beta"][:] = [float(st.beta) for st in stacks]
        start = np.concatenate(([0], np.cumsum(nl)[:-1]))
        rec["eps"][:] = eps_flat.ctypes.data + 8 * start.astype(np.uint64)
        wstart = np.concatenate(([0], np.cumsum(nw)[:-1]))
        rec["widths"][:] = np.where(nw > 0, w_flat.ctypes.data + 8 * wstart.astype(np.uint64),
                                    np.uint64(0))
        given = [i for i, m in enumerate(mus) if m is not None]
        if given:
            mu_flat = np.concatenate([mus[i] for i in given])
            keep.append(mu_flat)
            mstart = np.concatenate(([0], np.cumsum([len(mus[i]) for i in given])[:-1]))
            rec["mu"][given] = mu_flat.ctypes.data + 8 * mstart.astype(np.uint64)
    return rec.ctypes.data_as(C.POINTER(gfdtd_tmm_stack)), keep


def gfdtd_tmm(stacks: Sequence, omegas, stream=None):
    """Transfer-matrix (T, Gamma) of every stack (objects with eps, mu
    (or None), widths, beta) at every angular frequency: two complex arrays
    of shape (len(stacks), len(omegas))."""
    lib = load_library()
    arr, keep = _tmm_structs(stacks)
    om = np.ascontiguousarray(omegas, dtype=np.float64)
    n = C.c_size_t(0)
    _check(lib.gfdtd_tmm_workspace_bytes(arr, len(stacks), len(om), C.byref(n)))
    ws = _device_buffer(n.value)
    # (re, im) pairs written by the library are complex128 in memory order;
    # pinned (page-locked) host buffers let its device-to-host copy run at
    # full speed (torch caches them between calls)
    import torch
    shape = (len(stacks), len(om), 2)
    t = torch.empty(shape, dtype=torch.float64, pin_memory=True).numpy()
    g = torch.empty(shape, dtype=torch.float64, pin_memory=True).numpy()
    _check(lib.gfdtd_tmm(arr, len(stacks), om.ctypes.data_as(_PD), len(om),
                         C.c_void_p(ws.data_ptr()), n.value, _stream_handle(stream),
                         t.ctypes.data_as(_PD), g.ctypes.data_as(_PD)))
    del keep
    return t.view(np.complex128)[..., 0], g.view(np.complex128)[..., 0]


def gfdtd_tmm_kernel_ms() -> float:
    """Device time (ms) of the transfer-matrix kernel in this thread's last
    gfdtd_tmm call."""
    ms = C.c_double(0.0)
    _check(load_library().gfdtd_tmm_kernel_ms(C.byref(ms)))
    return ms.value


class Batch:
    """gfdtd_batch_prepare / run / collect / stats / destroy."""

    def __init__(self, problems: Sequence, steps=None, variant=GFDTD_VARIANT_AUTO,
                 cells_per_lane=0, block_steps=0, use_graph=-1, stream=None,
                 record_trace=True, fields=True, tile_waves=0, exchange_steps=0):
        import torch
        self._lib = load_library()
        self._ms, self._arr, self._st = _arrays(problems, steps)
        if record_trace:
            for i in range(len(self._ms)):
                self._arr[i].flags |= GFDTD_FLAG_RECORD_TRACE
        self._fields = fields
        self.stream = torch.cuda.current_stream() if stream is None else stream
        n = C.c_size_t(0)
        _check(self._lib.gfdtd_batch_workspace_bytes(
            self._arr, self._st.ctypes.data_as(_PI64), len(self._ms), C.byref(n)))
        self.workspace_bytes = n.value
        self._ws = _device_buffer(n.value)
        self._exec = _exec_struct(variant, cells_per_lane, block_steps, use_graph,
                                  tile_waves, exchange_steps)
        h = C.c_void_p(None)
        _check(self._lib.gfdtd_batch_prepare(
            self._arr, self._st.ctypes.data_as(_PI64), len(self._ms),
            C.byref(self._exec), C.c_void_p(self._ws.data_ptr()), n.value,
            _stream_handle(self.stream), C.byref(h)))
        self._h = h

    def run(self):
        _check(self._lib.gfdtd_batch_run(self._h))

    def collect(self) -> List[Dict[str, np.ndarray]]:
        outs = [_ResultBuffers(m, self._fields) for m in self._ms]
        res = (gfdtd_result * max(1, len(outs)))(*[o.struct for o in outs])
        _check(self._lib.gfdtd_batch_collect(self._h, res))
        for o, r in zip(outs, res):
            o.struct = r
        return [o.as_dict() for o in outs]

    def autotune(self, trial_blocks: int = 4) -> Dict[str, int]:
        """Pick cells per lane, steps per launch and waves per tile by
        timing trial launches on this batch (results do not depend on the
        choice)."""
        e = _exec_struct()
        _check(self._lib.gfdtd_batch_autotune(self._h, int(trial_blocks), C.byref(e)))
        return {"cells_per_lane": e.cells_per_lane, "block_steps": e.block_steps,
                "tile_waves": e.tile_waves, "exchange_steps": e.exchange_steps,
                "graph": e.use_graph}

    def stats(self) -> Dict[str, float]:
        s = gfdtd_stats()
        s.struct_size = C.sizeof(gfdtd_stats)
        _check(self._lib.gfdtd_batch_stats(self._h, C.byref(s)))
        return {k: getattr(s, k) for k, _ in gfdtd_stats._fields_ if k != "struct_size"}

    def close(self):
        if self._h:
            self._lib.gfdtd_batch_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """gfdtd_server_create / submit / progress / poll / destroy."""

    def __init__(self, pool_bytes: int, max_slots: int = 256, block_steps: int = 0,
                 stream=None, max_ahead: int = 0):
        import torch
        self._lib = load_library()
        self.stream = torch.cuda.current_stream() if stream is None else stream
        self._pool = _device_buffer(pool_bytes)
        cfg = gfdtd_server_config()
        cfg.struct_size = C.sizeof(gfdtd_server_config)
        cfg.max_slots = int(max_slots)
        cfg.block_steps = int(block_steps)
        cfg.max_ahead = int(max_ahead)
        cfg.pool = C.c_void_p(self._pool.data_ptr())
        cfg.pool_bytes = int(pool_bytes)
        cfg.stream = _stream_handle(self.stream)
        h = C.c_void_p(None)
        _check(self._lib.gfdtd_server_create(C.byref(cfg), C.byref(h)))
        self._h = h
        self._pending: Dict[int, _Marshalled] = {}

    def submit(self, problem, steps: Optional[int] = None, record_trace=False,
               keep_fields=False) -> int:
        m = _Marshalled(problem, steps)
        if record_trace:
            m.struct.flags |= GFDTD_FLAG_RECORD_TRACE
        if keep_fields:
            m.struct.flags |= GFDTD_FLAG_KEEP_FIELDS
        rid = C.c_uint64(0)
        _check(self._lib.gfdtd_server_submit(self._h, C.byref(m.struct), m.steps,
                                             C.byref(rid)))
        self._pending[rid.value] = m
        return rid.value

    def progress(self, max_blocks: int = 1):
        live, queued = C.c_int32(0), C.c_int32(0)
        _check(self._lib.gfdtd_server_progress(self._h, int(max_blocks),
                                               C.byref(live), C.byref(queued)))
        return live.value, queued.value

    def ready(self, rid: int) -> bool:
        st = self._lib.gfdtd_server_poll(self._h, C.c_uint64(rid), None)
        if st == GFDTD_E_NOT_READY:
            return False
        _check(st)
        return True

    def poll(self, rid: int) -> Optional[Dict[str, np.ndarray]]:
        """Results of a finished request (collected once), else None."""
        if not self.ready(rid):
            return None
        m = self._pending[rid]
        fields = bool(m.struct.flags & GFDTD_FLAG_KEEP_FIELDS)
        trace = bool(m.struct.flags & GFDTD_FLAG_RECORD_TRACE)
        out = _ResultBuffers(m, fields, trace)
        _check(self._lib.gfdtd_server_poll(self._h, C.c_uint64(rid), C.byref(out.struct)))
        del self._pending[rid]
        return out.as_dict()

    def close(self):
        if self._h:
            self._lib.gfdtd_server_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ 2D path

class _Marshalled2D:
    """A gfdtd2d_problem struct plus the numpy arrays it points into."""

    def __init__(self, p, steps: Optional[int] = None):
        self.nx, self.nz = int(p.nx), int(p.nz)
        self.eps = np.ascontiguousarray(p.eps_rest, dtype=np.float64)
        self.mu = np.ascontiguousarray(p.mu_rest, dtype=np.float64)
        prof = getattr(p, "src_profile", None)
        self.prof = None if prof is None else np.ascontiguousarray(prof, dtype=np.float64)
        self.px = np.ascontiguousarray(p.probe_x, dtype=np.int64)
        self.pz = np.ascontiguousarray(p.probe_z, dtype=np.int64)
        self.omegas = np.ascontiguousarray(p.omegas, dtype=np.float64)
        self.steps = int(p.steps if steps is None else steps)
        self.nprobe = len(self.px)
        self.nfreq = len(self.omegas)
        if len(self.pz) != self.nprobe:
            raise ValueError("probe_x and probe_z differ in length")
        s = gfdtd2d_problem()
        s.struct_size = C.sizeof(gfdtd2d_problem)
        s.pol = int(p.pol)
        s.precision = int(p.precision)
        s.abc = int(p.abc)
        s.flags = int(getattr(p, "flags", 0))
        s.nprobe = self.nprobe
        s.nfreq = self.nfreq
        s.nx, s.nz = self.nx, self.nz
        s.courant = float(p.courant)
        s.beta = float(p.beta)
        s.eps_rest = self.eps.ctypes.data_as(_PD)
        s.mu_rest = self.mu.ctypes.data_as(_PD)
        s.src_row = int(p.src_row)
        s.src_profile = None if self.prof is None else self.prof.ctypes.data_as(_PD)
        s.src_amp = float(p.pulse.amp)
        s.src_omega = float(p.pulse.omega)
        s.src_t0 = float(p.pulse.t0)
        s.src_tau = float(p.pulse.tau)
        s.src_phase = float(p.pulse.phase)
        s.src_t_off = float(p.pulse.t_off)
        s.probe_x = self.px.ctypes.data_as(_PI64) if self.nprobe else None
        s.probe_z = self.pz.ctypes.data_as(_PI64) if self.nprobe else None
        s.omegas = self.omegas.ctypes.data_as(_PD) if self.nfreq else None
        self.init = []
        for name in ("init_d", "init_b", "init_c"):
            a = getattr(p, name, None)
            if a is not None:
                a = np.ascontiguousarray(np.reshape(a, (self.nx * self.nz,)),
                                         dtype=np.float64)
                self.init.append(a)
                setattr(s, name, a.ctypes.data_as(_PD))
            else:
                setattr(s, name, None)
        self.struct = s


class _ResultBuffers2D:
    def __init__(self, m: _Marshalled2D, fields: bool = True, trace: bool = True):
        self.trace = np.zeros((m.nprobe, m.steps if trace else 0))
        self.dre = np.zeros((m.nprobe, m.nfreq))
        self.dim = np.zeros((m.nprobe, m.nfreq))
        shape = (m.nx, m.nz)
        self.f = {k: (np.zeros(shape) if fields else None) for k in ("d", "b", "c")}
        r = gfdtd2d_result()
        r.struct_size = C.sizeof(gfdtd2d_result)
        r.trace = self.trace.ctypes.data_as(_PD) if self.trace.size else None
        r.dft_re = self.dre.ctypes.data_as(_PD) if self.dre.size else None
        r.dft_im = self.dim.ctypes.data_as(_PD) if self.dim.size else None
        for k in ("d", "b", "c"):
            a = self.f[k]
            setattr(r, "final_" + k, None if a is None else a.ctypes.data_as(_PD))
        self.struct = r

    def as_dict(self) -> Dict[str, np.ndarray]:
        out = {"trace": self.trace, "dft": self.dre + 1j * self.dim,
               "status": int(self.struct.run_status),
               "steps_done": int(self.struct.steps_done)}
        for k, a in self.f.items():
            if a is not None:
                out[k] = a
        return out


def gfdtd2d_check(problem, steps: Optional[int] = None) -> float:
    """Validate a 2D problem and return the largest amplification factor
    per step of the pre-flight (raises GfdtdError on E_INVALID, and on
    E_UNSTABLE when the worst mode would grow more than tenfold over
    `steps`, default problem.steps)."""
    lib = load_library()
    m = _Marshalled2D(problem, steps)
    g = C.c_double(0.0)
    _check(lib.gfdtd2d_check(C.byref(m.struct), m.steps, C.byref(g)))
    return g.value


def gfdtd2d_workspace_bytes(problem, steps: Optional[int] = None) -> int:
    lib = load_library()
    m = _Marshalled2D(problem, steps)
    n = C.c_size_t(0)
    _check(lib.gfdtd2d_workspace_bytes(C.byref(m.struct), m.steps, C.byref(n)))
    return n.value


def gfdtd2d_solve(problem, steps: Optional[int] = None, stream=None,
                  fields: bool = True) -> Dict[str, np.ndarray]:
    """One 2D solve (synchronous).  Returns trace (nprobe, steps), dft
    (nprobe, nfreq) complex and the final d, b, c as (nx, nz) FP64 arrays."""
    lib = load_library()
    m = _Marshalled2D(problem, steps)
    m.struct.flags |= GFDTD_FLAG_RECORD_TRACE
    n = C.c_size_t(0)
    _check(lib.gfdtd2d_workspace_bytes(C.byref(m.struct), m.steps, C.byref(n)))
    ws = _device_buffer(n.value)
    out = _ResultBuffers2D(m, fields)
    _check(lib.gfdtd2d_solve(C.byref(m.struct), m.steps, C.c_void_p(ws.data_ptr()),
                             n.value, _stream_handle(stream), C.byref(out.struct)))
    return out.as_dict()


class Run2D:
    """gfdtd2d_prepare / run_pass / collect / get_stats / destroy."""

    def __init__(self, problem, steps=None, cells_per_lane=0, columns_per_wave=0,
                 block_steps=0, stream=None, record_trace=True, fields=True):
        import torch
        self._lib = load_library()
        self._m = _Marshalled2D(problem, steps)
        if record_trace:
            self._m.struct.flags |= GFDTD_FLAG_RECORD_TRACE
        self._fields = fields
        self.stream = torch.cuda.current_stream() if stream is None else stream
        n = C.c_size_t(0)
        _check(self._lib.gfdtd2d_workspace_bytes(C.byref(self._m.struct), self._m.steps,
                                                 C.byref(n)))
        self.workspace_bytes = n.value
        self._ws = _device_buffer(n.value)
        e = gfdtd2d_exec()
        e.struct_size = C.sizeof(gfdtd2d_exec)
        e.cells_per_lane = int(cells_per_lane)
        e.columns_per_wave = int(columns_per_wave)
        e.block_steps = int(block_steps)
        self._exec = e
        h = C.c_void_p(None)
        _check(self._lib.gfdtd2d_prepare(
            C.byref(self._m.struct), self._m.steps, C.byref(e),
            C.c_void_p(self._ws.data_ptr()), n.value, _stream_handle(self.stream),
            C.byref(h)))
        self._h = h

    def run(self):
        _check(self._lib.gfdtd2d_run_pass(self._h))

    def collect(self) -> Dict[str, np.ndarray]:
        out = _ResultBuffers2D(self._m, self._fields)
        _check(self._lib.gfdtd2d_collect(self._h, C.byref(out.struct)))
        return out.as_dict()

    def stats(self) -> Dict[str, float]:
        s = gfdtd2d_stats()
        s.struct_size = C.sizeof(gfdtd2d_stats)
        _check(self._lib.gfdtd2d_get_stats(self._h, C.byref(s)))
        return {k: getattr(s, k) for k, _ in gfdtd2d_stats._fields_
                if k not in ("struct_size", "reserved0")}

    def close(self):
        if self._h:
            self._lib.gfdtd2d_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
