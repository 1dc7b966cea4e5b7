"""Thin Python binding of libtl.so (include/tl.h).

Argument marshalling only: every step of a solve runs in the library's HIP
kernels.  Device buffers are PyTorch tensors (float64, [ny, nx, 2],
contiguous, on the current HIP device); streams are torch streams.  The
function names are those of the C ABI.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtl.so")

TL_OK, TL_PENDING, TL_E_INVAL, TL_E_NOMEM, TL_E_NOCONV, TL_E_DEVICE, TL_E_BUDGET, TL_E_NONFINITE = \
    0, 1, -1, -2, -3, -4, -5, -6
TL_FP64, TL_MIXED = 0, 1
TL_LOCAL_PCG, TL_LOCAL_EXACT = 0, 1

EXPORTS = (
    "tl_lattice_create", "tl_lattice_destroy", "tl_lattice_get_facts", "tl_solve",
    "tl_solve_batch", "tl_residual", "tl_server_create", "tl_submit", "tl_poll",
    "tl_server_destroy", "tl_strerror", "tl_solve_noalloc", "tl_tune", "tl_tune_lookup",
    "tl_tune_load", "tl_tune_save", "tl_tune_clear",
)

# Size of the fixed device array behind tl_solve_noalloc (TL_NOALLOC_SCRATCH_BYTES).
NOALLOC_SCRATCH_BYTES = 128 << 20


class LatticeDesc(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("ea", C.c_void_p),
                ("fixed", C.c_void_p), ("u_fixed", C.c_void_p),
                ("set_edge", C.c_int32), ("ptrs_on_device", C.c_int32)]


class TuneEntry(C.Structure):
    _fields_ = [("set_edge", C.c_int32), ("overlap", C.c_int32), ("inner_iters", C.c_int32),
                ("nx", C.c_int32), ("ny", C.c_int32), ("ms", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Trace(C.Structure):
    _fields_ = [("delta", C.c_void_p), ("kdiag", C.c_void_p), ("koff", C.c_void_p),
                ("force", C.c_void_p), ("coef", C.c_void_p),
                ("residual_history", C.c_void_p)]


class Opts(C.Structure):
    _fields_ = [("precision", C.c_int), ("rtol", C.c_double), ("max_iters", C.c_int32),
                ("inner_iters", C.c_int32), ("coarse_iters", C.c_int32),
                ("coarse_rtol", C.c_double), ("warm_start", C.c_int32),
                ("trace", C.POINTER(Trace)), ("profile", C.c_int32), ("overlap", C.c_int32),
                ("local_solve", C.c_int32)]


class Info(C.Structure):
    _fields_ = [("status", C.c_int), ("iters", C.c_int32), ("rel_res_l1", C.c_double),
                ("rel_res_l2", C.c_double), ("energy", C.c_double), ("ms", C.c_double),
                ("coarse_iters", C.c_int64), ("tile_ms", C.c_double), ("offdiag_ms", C.c_double),
                ("coarse_ms", C.c_double), ("tile_launches", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Facts(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("set_edge", C.c_int32),
                ("sets_x", C.c_int32), ("sets_y", C.c_int32), ("sets", C.c_int32),
                ("dof", C.c_int64), ("device_bytes", C.c_int64), ("solve_bytes", C.c_int64 * 2)]


_lib = None


def load():
    """Load libtl.so; raises if it has not been built (no fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_1208_4093_amd/build.sh")
        lib = C.CDLL(LIB_PATH)
        P = C.c_void_p
        lib.tl_lattice_create.argtypes = [C.POINTER(LatticeDesc), P, C.POINTER(P)]
        lib.tl_lattice_create.restype = C.c_int
        lib.tl_lattice_destroy.argtypes = [P]
        lib.tl_lattice_destroy.restype = None
        lib.tl_lattice_get_facts.argtypes = [P, C.POINTER(Facts)]
        lib.tl_lattice_get_facts.restype = C.c_int
        lib.tl_solve.argtypes = [P, P, P, C.POINTER(Opts), C.POINTER(Info), P]
        lib.tl_solve.restype = C.c_int
        lib.tl_solve_batch.argtypes = [C.c_int32, C.POINTER(P), C.POINTER(P), C.POINTER(P),
                                       C.POINTER(Opts), C.POINTER(Info), P]
        lib.tl_solve_batch.restype = C.c_int
        lib.tl_residual.argtypes = [P, P, P, P, C.POINTER(C.c_double), P]
        lib.tl_residual.restype = C.c_int
        lib.tl_server_create.argtypes = [C.c_size_t, C.c_int32, C.POINTER(P)]
        lib.tl_server_create.restype = C.c_int
        lib.tl_submit.argtypes = [P, P, P, P, C.POINTER(Opts), P, C.POINTER(C.c_uint64)]
        lib.tl_submit.restype = C.c_int
        lib.tl_poll.argtypes = [P, C.c_uint64, C.POINTER(Info)]
        lib.tl_poll.restype = C.c_int
        lib.tl_server_destroy.argtypes = [P]
        lib.tl_server_destroy.restype = None
        lib.tl_strerror.argtypes = [C.c_int]
        lib.tl_strerror.restype = C.c_char_p
        lib.tl_solve_noalloc.argtypes = [P, P, P, C.POINTER(Opts), C.POINTER(Info), P]
        lib.tl_solve_noalloc.restype = C.c_int
        lib.tl_tune.argtypes = [C.POINTER(LatticeDesc), P, C.POINTER(Opts), C.POINTER(TuneEntry), P]
        lib.tl_tune.restype = C.c_int
        lib.tl_tune_lookup.argtypes = [C.c_int32, C.c_int32, C.c_int, C.POINTER(TuneEntry)]
        lib.tl_tune_lookup.restype = C.c_int
        lib.tl_tune_load.argtypes = [C.c_char_p]
        lib.tl_tune_load.restype = C.c_int
        lib.tl_tune_save.argtypes = [C.c_char_p]
        lib.tl_tune_save.restype = C.c_int
        lib.tl_tune_clear.argtypes = []
        lib.tl_tune_clear.restype = C.c_int
        _lib = lib
    return _lib


class TLError(RuntimeError):
    def __init__(self, status, what):
        self.status = status
        super().__init__(f"{what}: {tl_strerror(status)} ({status})")


def tl_strerror(status: int) -> str:
    return load().tl_strerror(int(status)).decode()


def _stream_ptr(stream):
    """HIP stream handle: a torch stream, a raw handle, or None for torch's
    current stream (the null stream when no device is visible)."""
    if stream is None:
        import torch
        if not torch.cuda.is_available():
            return 0
        return torch.cuda.current_stream().cuda_stream
    return getattr(stream, "cuda_stream", stream)


def _dev_ptr(t, name, shape=None):
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float64 device tensor")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return t.data_ptr()


class Lattice:
    """Owning handle of a tl_lattice."""

    def __init__(self, handle, nx, ny):
        self.handle = handle
        self.nx, self.ny = nx, ny
        f = self.facts()
        self.set_edge, self.sets_x, self.sets_y, self.sets = (f["set_edge"], f["sets_x"],
                                                              f["sets_y"], f["sets"])
        self.dof, self.device_bytes = f["dof"], f["device_bytes"]
        self.solve_bytes = f["solve_bytes"]

    def facts(self):
        """tl_lattice_get_facts now (device_bytes grows as solves add state)."""
        f = Facts()
        st = load().tl_lattice_get_facts(self.handle, C.byref(f))
        if st != TL_OK:
            raise TLError(st, "tl_lattice_get_facts")
        return dict(set_edge=f.set_edge, sets_x=f.sets_x, sets_y=f.sets_y, sets=f.sets,
                    dof=f.dof, device_bytes=f.device_bytes,
                    solve_bytes=(f.solve_bytes[0], f.solve_bytes[1]))

    def close(self):
        if self.handle:
            load().tl_lattice_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _lattice_desc(nx, ny, ea, fixed, u_fixed, set_edge):
    """The tl_lattice_desc of host numpy arrays or device torch tensors, and
    the arrays it points into (to be kept alive for the call)."""
    keep = []
    on_dev = None

    def ptr(a, dtype, shape, name):
        nonlocal on_dev
        if a is None:
            return None
        try:
            import torch
            is_t = isinstance(a, torch.Tensor)
        except ImportError:
            is_t = False
        if is_t:
            dev = a.is_cuda
            if tuple(a.shape) != shape or not a.is_contiguous():
                raise ValueError(f"{name}: expected contiguous {shape}")
            keep.append(a)
            p = a.data_ptr()
        else:
            dev = False
            arr = np.ascontiguousarray(a, dtype=dtype)
            if arr.shape != shape:
                raise ValueError(f"{name}: expected shape {shape}, got {arr.shape}")
            keep.append(arr)
            p = arr.ctypes.data
        if on_dev is None:
            on_dev = dev
        elif on_dev != dev:
            raise ValueError("ea, fixed and u_fixed must all be on the host or all on the device")
        return p

    d = LatticeDesc()
    d.nx, d.ny = int(nx), int(ny)
    d.ea = ptr(ea, np.float32, (3, ny, nx), "ea")
    d.fixed = ptr(fixed, np.uint8, (ny, nx), "fixed")
    d.u_fixed = ptr(u_fixed, np.float64, (ny, nx, 2), "u_fixed")
    d.set_edge = int(set_edge)
    d.ptrs_on_device = 1 if on_dev else 0
    return d, keep


def tl_lattice_create(nx, ny, ea=None, fixed=None, u_fixed=None, set_edge=0, stream=None):
    """Create a lattice from host numpy arrays (ea float32 [3, ny, nx], fixed
    uint8 [ny, nx], u_fixed float64 [ny, nx, 2]) or device torch tensors."""
    d, keep = _lattice_desc(nx, ny, ea, fixed, u_fixed, set_edge)
    h = C.c_void_p()
    st = load().tl_lattice_create(C.byref(d), C.c_void_p(_stream_ptr(stream)), C.byref(h))
    if st != TL_OK:
        raise TLError(st, "tl_lattice_create")
    return Lattice(h, nx, ny)


def make_opts(precision=TL_FP64, rtol=1e-8, max_iters=0, inner_iters=0, coarse_iters=0,
              coarse_rtol=0.0, warm_start=False, trace=None, profile=False, overlap=0,
              local_solve=0):
    o = Opts()
    o.precision = int(precision)
    o.rtol = float(rtol)
    o.max_iters = int(max_iters)
    o.inner_iters = int(inner_iters)
    o.coarse_iters = int(coarse_iters)
    o.coarse_rtol = float(coarse_rtol)
    o.warm_start = 1 if warm_start else 0
    o.trace = C.pointer(trace) if trace is not None else C.POINTER(Trace)()
    o.profile = int(profile)
    o.overlap = int(overlap)
    o.local_solve = int(local_solve)
    return o


def make_trace(delta=None, kdiag=None, koff=None, force=None, coef=None, residual_history=None):
    tr = Trace()
    for name, t in (("delta", delta), ("kdiag", kdiag), ("koff", koff), ("force", force),
                    ("coef", coef), ("residual_history", residual_history)):
        setattr(tr, name, None if t is None else _dev_ptr(t, name))
    return tr


def tl_solve(lat: Lattice, f, u, stream=None, check=True, **opts):
    """Solve K u = f on the device; u is written in place.  Returns the
    tl_info as a dict (raises TLError on failure when check is set)."""
    shape = (lat.ny, lat.nx, 2)
    o = make_opts(**opts)
    info = Info()
    st = load().tl_solve(lat.handle, C.c_void_p(_dev_ptr(f, "f", shape)),
                         C.c_void_p(_dev_ptr(u, "u", shape)), C.byref(o), C.byref(info),
                         C.c_void_p(_stream_ptr(stream)))
    if check and st != TL_OK:
        raise TLError(st, "tl_solve")
    out = info.as_dict()
    out["status"] = st
    return out


def tl_solve_noalloc(lat: Lattice, f, u, stream=None, check=True, **opts):
    """tl_solve with the solve state in the library's fixed device array (no
    allocation).  Same arguments and result as tl_solve."""
    shape = (lat.ny, lat.nx, 2)
    o = make_opts(**opts)
    info = Info()
    st = load().tl_solve_noalloc(lat.handle, C.c_void_p(_dev_ptr(f, "f", shape)),
                                 C.c_void_p(_dev_ptr(u, "u", shape)), C.byref(o), C.byref(info),
                                 C.c_void_p(_stream_ptr(stream)))
    if check and st != TL_OK:
        raise TLError(st, "tl_solve_noalloc")
    out = info.as_dict()
    out["status"] = st
    return out


def tl_solve_batch(lats, fs, us, stream=None, check=True, **opts):
    n = len(lats)
    P = C.c_void_p
    hl = (P * n)(*[l.handle for l in lats])
    hf = (P * n)(*[_dev_ptr(f, "f", (l.ny, l.nx, 2)) for l, f in zip(lats, fs)])
    hu = (P * n)(*[_dev_ptr(u, "u", (l.ny, l.nx, 2)) for l, u in zip(lats, us)])
    o = make_opts(**opts)
    infos = (Info * n)()
    st = load().tl_solve_batch(n, hl, hf, hu, C.byref(o), infos, C.c_void_p(_stream_ptr(stream)))
    if check and st != TL_OK:
        raise TLError(st, "tl_solve_batch")
    return st, [i.as_dict() for i in infos]


def tl_residual(lat: Lattice, f, u, r=None, stream=None):
    """(R1, R2, energy) of u, and r = f - K u into r when given."""
    shape = (lat.ny, lat.nx, 2)
    out = (C.c_double * 3)()
    st = load().tl_residual(lat.handle, C.c_void_p(_dev_ptr(f, "f", shape)),
                            C.c_void_p(_dev_ptr(u, "u", shape)),
                            C.c_void_p(None if r is None else _dev_ptr(r, "r", shape)),
                            out, C.c_void_p(_stream_ptr(stream)))
    if st != TL_OK:
        raise TLError(st, "tl_residual")
    return out[0], out[1], out[2]


class Server:
    def __init__(self, handle):
        self.handle = handle
        self._keep = {}

    def close(self):
        if self.handle:
            load().tl_server_destroy(self.handle)
            self.handle = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def tl_server_create(hbm_budget_bytes: int, max_slots: int) -> Server:
    h = C.c_void_p()
    st = load().tl_server_create(C.c_size_t(int(hbm_budget_bytes)), int(max_slots), C.byref(h))
    if st != TL_OK:
        raise TLError(st, "tl_server_create")
    return Server(h)


def tl_submit(srv: Server, lat: Lattice, f, u, stream=None, **opts) -> int:
    """Queue a solve; its kernels wait for the work enqueued on `stream` (torch's
    current stream by default) before the call."""
    shape = (lat.ny, lat.nx, 2)
    o = make_opts(**opts)
    ticket = C.c_uint64()
    st = load().tl_submit(srv.handle, lat.handle, C.c_void_p(_dev_ptr(f, "f", shape)),
                          C.c_void_p(_dev_ptr(u, "u", shape)), C.byref(o),
                          C.c_void_p(_stream_ptr(stream)), C.byref(ticket))
    if st != TL_OK:
        raise TLError(st, "tl_submit")
    srv._keep[ticket.value] = (lat, f, u)
    return ticket.value


def tl_poll(srv: Server, ticket: int):
    """(status, info dict); status TL_PENDING until the request finished."""
    info = Info()
    st = load().tl_poll(srv.handle, C.c_uint64(ticket), C.byref(info))
    if st != TL_PENDING:
        srv._keep.pop(ticket, None)
    return st, info.as_dict()


# ---------------------------------------------------------------- autotuning

def tl_tune(nx, ny, f, ea=None, fixed=None, u_fixed=None, stream=None, check=True, **opts):
    """Measure launch choices for the lattice's shape and precision (opts as
    for tl_solve; overlap and inner_iters are searched) and record the
    fastest under the shape's key.  Returns the chosen entry as a dict."""
    d, keep = _lattice_desc(nx, ny, ea, fixed, u_fixed, 0)
    o = make_opts(**opts)
    e = TuneEntry()
    st = load().tl_tune(C.byref(d), C.c_void_p(_dev_ptr(f, "f", (ny, nx, 2))), C.byref(o),
                        C.byref(e), C.c_void_p(_stream_ptr(stream)))
    del keep
    if check and st != TL_OK:
        raise TLError(st, "tl_tune")
    out = e.as_dict()
    out["status"] = st
    return out


def tl_tune_lookup(nx, ny, precision=TL_FP64):
    """The table's entry for a shape and precision, or None."""
    e = TuneEntry()
    st = load().tl_tune_lookup(int(nx), int(ny), int(precision), C.byref(e))
    if st != TL_OK:
        raise TLError(st, "tl_tune_lookup")
    return e.as_dict() if e.set_edge else None


def tl_tune_load(path):
    st = load().tl_tune_load(os.fsencode(path))
    if st != TL_OK:
        raise TLError(st, "tl_tune_load")


def tl_tune_save(path):
    st = load().tl_tune_save(os.fsencode(path))
    if st != TL_OK:
        raise TLError(st, "tl_tune_save")


def tl_tune_clear():
    load().tl_tune_clear()
