"""ctypes binding of libbinning.so (include/binning.h).

Argument marshalling only: every step of the binning runs in the HIP
library.  PyTorch supplies device memory and streams; a tensor argument is
passed as its data pointer and a stream as its raw hipStream_t.

The library must have been built in-tree (``python -m
paper_2310_02926_amd.build``); loading fails loudly otherwise.  torch is
imported before the library is loaded so that the process holds a single HIP
runtime (torch's, which has the same soname as the system one).
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_int, c_int32, c_int64, c_size_t, c_uint32, c_uint64, c_void_p
from typing import Dict, List, Optional, Sequence

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libbinning.so")

BIN_OK, BIN_ERR_INVALID_ARG, BIN_ERR_UNSUPPORTED, BIN_ERR_OOM, BIN_ERR_DEVICE = 0, -1, -2, -3, -4
BIN_ERR_ADMISSION, BIN_ERR_TIMEOUT, BIN_ERR_NOT_FOUND = -5, -6, -7
BIN_F32, BIN_F64 = 0, 1
COUNT, SUM, MIN, MAX, AVG = 1, 2, 4, 8, 16
OPS_ALL = 31
PREC_PLAIN, PREC_F64, PREC_COMP = 0x100, 0x200, 0x400
STRAT_AUTO, STRAT_GLOBAL, STRAT_LDS, STRAT_PART = -1, 0, 1, 2
MAX_ATTRS = 16

#: Every function declared in include/binning.h.
EXPORTS = (
    "bin_particles", "bin_particles_noalloc", "bin_validate", "bin_particles_nd", "bin_validate_nd", "bin_particles_async", "bin_particles_batched", "bin_particles_multi", "bin_graph_create", "bin_graph_create_multi", "bin_graph_launch",
    "bin_graph_destroy", "bin_autotune", "bin_status_string", "bin_last_error_message",
    "bin_stream_status", "bin_release_workspace", "bin_version", "bin_timing_enable", "bin_timing_read",
    "bin_timing_report",
    "bin_describe_plan", "bin_describe_plan_on", "bin_set_plan_override", "bin_set_tuning", "bin_copy_to_host", "binsrv_create", "binsrv_submit", "binsrv_wait", "binsrv_release",
    "binsrv_get_stats", "binsrv_destroy",
)


class Columns(ctypes.Structure):
    _fields_ = [("cols", POINTER(c_void_p)), ("ncols", c_int32), ("dtype", c_int32)]


class Output(ctypes.Structure):
    _fields_ = [("count", c_void_p), ("sum", POINTER(c_void_p)), ("min", POINTER(c_void_p)),
                ("max", POINTER(c_void_p)), ("avg", POINTER(c_void_p))]


class Request(ctypes.Structure):
    _fields_ = [("coords", Columns), ("attrs", Columns), ("n", c_int64), ("axes", c_int32 * 2),
                ("bounds", c_double * 4), ("nx", c_int32), ("ny", c_int32), ("ops", c_uint32),
                ("out", Output)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("budget_bytes", c_uint64), ("n_slots", c_int32), ("max_batch", c_int32),
                ("device", c_int32), ("reserved", c_int32)]


class ServerRequest(ctypes.Structure):
    _fields_ = [("coords", Columns), ("attrs", Columns), ("n", c_int64), ("axes", c_int32 * 2),
                ("bounds", c_double * 4), ("nx", c_int32), ("ny", c_int32), ("ops", c_uint32),
                ("producer_stream", c_void_p)]


class GridSpec(ctypes.Structure):
    _fields_ = [("axes", c_int32 * 2), ("bounds", c_double * 4), ("nx", c_int32), ("ny", c_int32),
                ("ops", c_uint32), ("out", Output)]


class Result(ctypes.Structure):
    _fields_ = [("status", c_int32), ("k", c_int32), ("count", c_void_p),
                ("sum", c_void_p * MAX_ATTRS), ("min", c_void_p * MAX_ATTRS),
                ("max", c_void_p * MAX_ATTRS), ("avg", c_void_p * MAX_ATTRS),
                ("submit_to_done_ms", c_double), ("queue_ms", c_double)]


class ServerStats(ctypes.Structure):
    _fields_ = [(n, c_uint64) for n in ("submitted", "completed", "failed", "released", "batches",
                                        "in_flight", "queued", "bytes_in_use", "peak_bytes")]


class BinError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{status_string(status)}: {message}")
        self.status = status


_lib = None


def lib() -> ctypes.CDLL:
    """Load libbinning.so once (after torch, so one HIP runtime is mapped)."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  (load torch's HIP runtime first)
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2310_02926_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    sig = {
        "bin_particles": (c_int, [POINTER(Columns), POINTER(Columns), c_int64, POINTER(c_int32),
                                  POINTER(c_double), c_int32, c_int32, c_uint32, POINTER(Output), c_void_p]),
        "bin_particles_noalloc": (c_int, [POINTER(Columns), POINTER(Columns), c_int64, POINTER(c_int32),
                                          POINTER(c_double), c_int32, c_int32, c_uint32, POINTER(Output),
                                          c_void_p]),
        "bin_validate": (c_int, [POINTER(Columns), POINTER(Columns), c_int64, POINTER(c_int32),
                                 POINTER(c_double), c_int32, c_int32, c_uint32, POINTER(Output)]),
        "bin_particles_nd": (c_int, [POINTER(Columns), POINTER(Columns), c_int64, c_int32, POINTER(c_int32),
                                     POINTER(c_double), POINTER(c_int32), c_uint32, POINTER(Output), c_void_p]),
        "bin_validate_nd": (c_int, [POINTER(Columns), POINTER(Columns), c_int64, c_int32, POINTER(c_int32),
                                    POINTER(c_double), POINTER(c_int32), c_uint32, POINTER(Output)]),
        "bin_particles_async": (c_int, [POINTER(Columns), POINTER(Columns), c_int64, POINTER(c_int32),
                                        POINTER(c_double), c_int32, c_int32, c_uint32, POINTER(Output), c_void_p,
                                        c_void_p]),
        "bin_particles_batched": (c_int, [POINTER(Request), c_int32, c_void_p]),
        "bin_particles_multi": (c_int, [POINTER(Columns), POINTER(Columns), c_int64, POINTER(GridSpec), c_int32,
                                        c_void_p]),
        "bin_graph_create": (c_int, [POINTER(Request), c_int32, POINTER(c_void_p)]),
        "bin_graph_create_multi": (c_int, [POINTER(Columns), POINTER(Columns), c_int64, POINTER(GridSpec), c_int32,
                                           POINTER(c_void_p)]),
        "bin_graph_launch": (c_int, [c_void_p, c_void_p]),
        "bin_graph_destroy": (c_int, [c_void_p]),
        "bin_autotune": (c_int, [POINTER(Request), c_int32]),
        "bin_status_string": (c_char_p, [c_int]),
        "bin_last_error_message": (c_char_p, []),
        "bin_stream_status": (c_int, [c_void_p]),
        "bin_release_workspace": (c_int, []),
        "bin_version": (c_char_p, []),
        "bin_timing_enable": (c_int, [c_int]),
        "bin_timing_read": (c_int, [POINTER(c_int64), POINTER(c_double)]),
        "bin_timing_report": (c_int, [c_char_p, c_size_t]),
        "bin_describe_plan": (c_int, [POINTER(Request), c_char_p, c_size_t]),
        "bin_describe_plan_on": (c_int, [POINTER(Request), c_int32, c_int64, c_int64, c_char_p, c_size_t]),
        "bin_set_plan_override": (c_int, [c_int32, c_int32, c_int32]),
        "bin_set_tuning": (c_int, [c_int32, c_int64]),
        "bin_copy_to_host": (c_int, [c_void_p, c_void_p, c_size_t]),
        "binsrv_create": (c_int, [POINTER(ServerConfig), POINTER(c_void_p)]),
        "binsrv_submit": (c_int, [c_void_p, POINTER(ServerRequest), POINTER(c_uint64)]),
        "binsrv_wait": (c_int, [c_void_p, c_uint64, c_int64, POINTER(Result)]),
        "binsrv_release": (c_int, [c_void_p, c_uint64]),
        "binsrv_get_stats": (c_int, [c_void_p, POINTER(ServerStats)]),
        "binsrv_destroy": (c_int, [c_void_p]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def status_string(status: int) -> str:
    return lib().bin_status_string(status).decode()


def last_error() -> str:
    return lib().bin_last_error_message().decode()


def check(status: int) -> int:
    if status != BIN_OK:
        raise BinError(status, last_error())
    return status


# ---------------------------------------------------------------------------
# Marshalling helpers
# ---------------------------------------------------------------------------

def _ptr(x) -> Optional[int]:
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return int(x.data_ptr())


def _dtype_code(t) -> int:
    import torch
    if isinstance(t, int):
        return t
    if t.dtype == torch.float32:
        return BIN_F32
    if t.dtype == torch.float64:
        return BIN_F64
    raise TypeError(f"unsupported column dtype {t.dtype}")


def _ptr_array(items) -> Optional[ctypes.Array]:
    if items is None:
        return None
    arr = (c_void_p * max(len(items), 1))()
    for i, it in enumerate(items):
        arr[i] = _ptr(it)
    return arr


def columns(cols: Sequence, dtype: Optional[int] = None):
    """A Columns record (and the pointer array it references) for tensors or
    raw pointers; ``dtype`` is required for raw pointers."""
    arr = _ptr_array(list(cols))
    code = dtype if dtype is not None else (_dtype_code(cols[0]) if len(cols) else BIN_F32)
    return Columns(ctypes.cast(arr, POINTER(c_void_p)), len(cols), code), arr


def output(count=None, sums=None, mins=None, maxs=None, avgs=None):
    keep = [_ptr_array(x) for x in (sums, mins, maxs, avgs)]
    cast = [ctypes.cast(a, POINTER(c_void_p)) if a is not None else None for a in keep]
    return Output(_ptr(count), *cast), keep


def _stream_handle(stream) -> Optional[int]:
    if stream is None:
        import torch
        return int(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)


# ---------------------------------------------------------------------------
# Entry points (same names as the C ABI)
# ---------------------------------------------------------------------------

def bin_particles(coords, attrs, n: int, axes, bounds, nx: int, ny: int, ops: int, out: Dict,
                  stream=None, coord_dtype=None, attr_dtype=None) -> None:
    """Enqueue one binning request.  ``coords``/``attrs``: sequences of CUDA
    tensors (or raw device pointers with ``*_dtype``); ``out``: dict with
    optional 'count' and lists 'sum'/'min'/'max'/'avg' of tensors/pointers;
    ``bounds`` None asks for bounds computed on the fly."""
    c, ck = columns(coords, coord_dtype)
    a, ak = columns(attrs, attr_dtype) if attrs is not None else (None, None)
    o, ok = output(out.get("count"), out.get("sum"), out.get("min"), out.get("max"), out.get("avg"))
    ax = (c_int32 * 2)(*axes)
    bd = (c_double * 4)(*bounds) if bounds is not None else None
    st = lib().bin_particles(ctypes.byref(c), ctypes.byref(a) if a is not None else None, n, ax, bd,
                             nx, ny, ops, ctypes.byref(o), _stream_handle(stream))
    check(st)


class Call:
    """One request (bin_particles) marshalled once and enqueued many times,
    as a simulation bins its particles every step: each launch passes the
    prepared records and only the stream handle is looked up again."""

    def __init__(self, coords, attrs, n: int, axes, bounds, nx: int, ny: int, ops: int, out: Dict,
                 coord_dtype=None, attr_dtype=None):
        self._c, self._ck = columns(coords, coord_dtype)
        self._a, self._ak = columns(attrs, attr_dtype) if attrs is not None else (None, None)
        self._o, self._ok = output(out.get("count"), out.get("sum"), out.get("min"), out.get("max"), out.get("avg"))
        self._args = (ctypes.byref(self._c), ctypes.byref(self._a) if self._a is not None else None, n,
                      (c_int32 * 2)(*axes), (c_double * 4)(*bounds) if bounds is not None else None, nx, ny, ops,
                      ctypes.byref(self._o))
        self._fn = lib().bin_particles

    def launch(self, stream=None) -> None:
        check(self._fn(*self._args, _stream_handle(stream)))


def bin_particles_noalloc(coords, attrs, n: int, axes, bounds, nx: int, ny: int, ops: int, out: Dict,
                          stream=None, coord_dtype=None, attr_dtype=None) -> None:
    """bin_particles with the library's scratch in its fixed per-GPU array
    (no device allocation); arguments as bin_particles."""
    c, ck = columns(coords, coord_dtype)
    a, ak = columns(attrs, attr_dtype) if attrs is not None else (None, None)
    o, ok = output(out.get("count"), out.get("sum"), out.get("min"), out.get("max"), out.get("avg"))
    ax = (c_int32 * 2)(*axes)
    bd = (c_double * 4)(*bounds) if bounds is not None else None
    st = lib().bin_particles_noalloc(ctypes.byref(c), ctypes.byref(a) if a is not None else None, n, ax, bd,
                                     nx, ny, ops, ctypes.byref(o), _stream_handle(stream))
    check(st)


def _nd_args(axes, bounds, dims):
    d = len(axes)
    ax = (c_int32 * d)(*axes)
    dm = (c_int32 * len(dims))(*dims)
    bd = (c_double * (2 * d))(*bounds) if bounds is not None else None
    return d, ax, bd, dm


def bin_particles_nd(coords, attrs, n: int, axes, bounds, dims, ops: int, out: Dict, stream=None,
                     coord_dtype=None, attr_dtype=None) -> None:
    """Enqueue one request on a mesh of len(axes) = 1, 2 or 3 axes;
    ``bounds`` = (lo0, hi0, lo1, hi1, ...) or None; ``dims`` = bins per
    axis.  Output grids hold prod(dims) elements, axis 0 fastest."""
    c, ck = columns(coords, coord_dtype)
    a, ak = columns(attrs, attr_dtype) if attrs is not None else (None, None)
    o, ok = output(out.get("count"), out.get("sum"), out.get("min"), out.get("max"), out.get("avg"))
    d, ax, bd, dm = _nd_args(axes, bounds, dims)
    check(lib().bin_particles_nd(ctypes.byref(c), ctypes.byref(a) if a is not None else None, n, d, ax, bd, dm,
                                 ops, ctypes.byref(o), _stream_handle(stream)))


def bin_validate_nd(coords, attrs, n, axes, bounds, dims, ops, out, coord_dtype=None, attr_dtype=None,
                    ndim=None) -> int:
    """Host-only argument check of bin_particles_nd; returns the status.
    ``ndim`` overrides len(axes) (to test the ndim check itself)."""
    c, ck = columns(coords, coord_dtype)
    a, ak = columns(attrs, attr_dtype) if attrs is not None else (None, None)
    o, ok = output(out.get("count"), out.get("sum"), out.get("min"), out.get("max"), out.get("avg"))
    d, ax, bd, dm = _nd_args(axes, bounds, dims)
    return lib().bin_validate_nd(ctypes.byref(c), ctypes.byref(a) if a is not None else None, n,
                                 d if ndim is None else ndim, ax, bd, dm, ops, ctypes.byref(o))


def alloc_outputs_nd(attrs, dims, ops: int, device) -> Dict:
    """Output grids shaped dims reversed ([d2][d1][d0]) for bin_particles_nd."""
    nb = 1
    for v in dims:
        nb *= int(v)
    out = alloc_outputs(attrs, nb, 1, ops, device)
    shape = tuple(int(v) for v in reversed(dims))
    return {k: (v.view(shape) if not isinstance(v, list) else [t.view(shape) for t in v]) for k, v in out.items()}


def bin_particles_async(coords, attrs, n: int, axes, bounds, nx: int, ny: int, ops: int, out: Dict,
                        src_stream=None, bin_stream=None, coord_dtype=None, attr_dtype=None) -> None:
    """Deep-copy the request's columns on src_stream and bin the copy on
    bin_stream (the asynchronous in situ mode); see the C header."""
    c, ck = columns(coords, coord_dtype)
    a, ak = columns(attrs, attr_dtype) if attrs is not None else (None, None)
    o, ok = output(out.get("count"), out.get("sum"), out.get("min"), out.get("max"), out.get("avg"))
    ax = (c_int32 * 2)(*axes)
    bd = (c_double * 4)(*bounds) if bounds is not None else None
    check(lib().bin_particles_async(ctypes.byref(c), ctypes.byref(a) if a is not None else None, n, ax, bd, nx, ny,
                                    ops, ctypes.byref(o), _stream_handle(src_stream), _stream_handle(bin_stream)))


def bin_validate(coords, attrs, n, axes, bounds, nx, ny, ops, out, coord_dtype=None, attr_dtype=None) -> int:
    """Host-only argument check; returns the status (no exception)."""
    c, ck = columns(coords, coord_dtype)
    a, ak = columns(attrs, attr_dtype) if attrs is not None else (None, None)
    o, ok = output(out.get("count"), out.get("sum"), out.get("min"), out.get("max"), out.get("avg"))
    ax = (c_int32 * 2)(*axes)
    bd = (c_double * 4)(*bounds) if bounds is not None else None
    return lib().bin_validate(ctypes.byref(c), ctypes.byref(a) if a is not None else None, n, ax, bd,
                              nx, ny, ops, ctypes.byref(o))


def output_dtypes(attr_is_f64: bool, ops: int):
    """(sum/avg dtype, min/max dtype) as torch dtypes, per the header's rules."""
    import torch
    mm = torch.float64 if attr_is_f64 else torch.float32
    sa = torch.float32 if (not attr_is_f64 and ops & PREC_PLAIN) else torch.float64
    return sa, mm


def alloc_outputs(attrs, nx: int, ny: int, ops: int, device) -> Dict:
    """Allocate (uninitialised) output grids for a request with torch."""
    import torch
    k = len(attrs) if attrs is not None else 0
    af64 = k > 0 and attrs[0].dtype == torch.float64
    sa, mm = output_dtypes(af64, ops)
    out = {}
    if ops & COUNT:
        out["count"] = torch.empty((ny, nx), dtype=torch.int32, device=device)  # holds uint32 bits
    for key, bit, dt in (("sum", SUM, sa), ("min", MIN, mm), ("max", MAX, mm), ("avg", AVG, sa)):
        if ops & bit:
            out[key] = [torch.empty((ny, nx), dtype=dt, device=device) for _ in range(k)]
    return out


def bin_particles_alloc(coords, attrs, axes=(0, 1), bounds=(0.0, 1.0, 0.0, 1.0), nx: int = 64,
                        ny: int = 64, ops: int = OPS_ALL, stream=None) -> Dict:
    """Allocate outputs on the columns' device and enqueue bin_particles."""
    n = int(coords[0].numel())
    out = alloc_outputs(attrs, nx, ny, ops, coords[0].device)
    bin_particles(coords, attrs, n, axes, bounds, nx, ny, ops, out, stream)
    return out


def request(coords, attrs, n, axes, bounds, nx, ny, ops, out):
    """A Request record plus the ctypes objects it references (keep both)."""
    c, ck = columns(coords)
    a, ak = columns(attrs) if attrs else (Columns(None, 0, BIN_F32), None)
    o, ok = output(out.get("count"), out.get("sum"), out.get("min"), out.get("max"), out.get("avg"))
    r = Request(c, a, n, (c_int32 * 2)(*axes), (c_double * 4)(*bounds), nx, ny, ops, o)
    return r, (ck, ak, ok)


def request_array(reqs: Sequence[Dict]):
    """A ctypes array of Request records from dicts with the keyword
    arguments of bin_particles (coords, attrs, n, axes, bounds, nx, ny, ops,
    out), plus the objects they reference (keep both alive)."""
    arr = (Request * max(len(reqs), 1))()
    keep = []
    for i, r in enumerate(reqs):
        rec, k = request(r["coords"], r.get("attrs") or [], r["n"], r.get("axes", (0, 1)),
                         r.get("bounds", (0.0, 1.0, 0.0, 1.0)), r["nx"], r["ny"], r["ops"], r["out"])
        arr[i] = rec
        keep.append(k)
    return arr, keep


def bin_particles_batched(reqs: Sequence[Dict], stream=None) -> None:
    """Enqueue a batch of independent requests (see request_array)."""
    arr, keep = request_array(reqs)
    check(lib().bin_particles_batched(arr, len(reqs), _stream_handle(stream)))


def bin_autotune(reqs: Sequence[Dict]) -> None:
    """Time candidate configurations for these request shapes (overwrites
    their outputs; synchronises a private stream) and remember the best."""
    arr, keep = request_array(reqs)
    check(lib().bin_autotune(arr, len(reqs)))


def grid_specs(grids: Sequence[Dict]):
    """A ctypes array of GridSpec records from dicts with keys axes, bounds,
    nx, ny, ops, out (as bin_particles), plus the objects they reference."""
    arr = (GridSpec * max(len(grids), 1))()
    keep = []
    for i, g in enumerate(grids):
        out = g["out"]
        o, ok = output(out.get("count"), out.get("sum"), out.get("min"), out.get("max"), out.get("avg"))
        arr[i] = GridSpec((c_int32 * 2)(*g["axes"]), (c_double * 4)(*g["bounds"]), g["nx"], g["ny"], g["ops"], o)
        keep.append(ok)
    return arr, keep


def bin_particles_multi(coords, attrs, n: int, grids: Sequence[Dict], stream=None, coord_dtype=None,
                        attr_dtype=None) -> None:
    """Enqueue one binning of the table per grid spec (see grid_specs)."""
    c, ck = columns(coords, coord_dtype)
    a, ak = columns(attrs, attr_dtype) if attrs else (None, None)
    arr, keep = grid_specs(grids)
    check(lib().bin_particles_multi(ctypes.byref(c), ctypes.byref(a) if a is not None else None, n, arr,
                                    len(grids), _stream_handle(stream)))


class Multi:
    """A multi-grid call (bin_particles_multi) marshalled once and enqueued
    many times, as a simulation does every step."""

    def __init__(self, coords, attrs, n: int, grids: Sequence[Dict], coord_dtype=None, attr_dtype=None):
        self._c, self._ck = columns(coords, coord_dtype)
        self._a, self._ak = columns(attrs, attr_dtype) if attrs else (None, None)
        self._arr, self._keep = grid_specs(grids)
        self.n = n
        self.ngrids = len(grids)

    def launch(self, stream=None) -> None:
        check(lib().bin_particles_multi(ctypes.byref(self._c),
                                        ctypes.byref(self._a) if self._a is not None else None, self.n, self._arr,
                                        self.ngrids, _stream_handle(stream)))


class Batch:
    """Requests marshalled once and enqueued many times, as one batch
    (bin_particles_batched) or one request at a time (bin_particles)."""

    def __init__(self, reqs: Sequence[Dict]):
        self.arr, self._keep = request_array(reqs)
        self.n = len(reqs)

    def launch(self, stream=None) -> None:
        check(lib().bin_particles_batched(self.arr, self.n, _stream_handle(stream)))

    def launch_one(self, i: int, stream=None) -> None:
        r = self.arr[i]
        check(lib().bin_particles(ctypes.byref(r.coords), ctypes.byref(r.attrs), r.n, r.axes, r.bounds, r.nx,
                                  r.ny, r.ops, ctypes.byref(r.out), _stream_handle(stream)))


class BinGraph:
    """A captured batch (or, with multi(), a captured multi-grid call):
    create once, launch many times, destroy."""

    def __init__(self, reqs: Sequence[Dict]):
        arr, self._keep = request_array(reqs)
        h = c_void_p()
        check(lib().bin_graph_create(arr, len(reqs), ctypes.byref(h)))
        self._h = h

    @classmethod
    def multi(cls, coords, attrs, n: int, grids: Sequence[Dict], coord_dtype=None, attr_dtype=None) -> "BinGraph":
        """bin_graph_create_multi: what bin_particles_multi enqueues, captured."""
        g = cls.__new__(cls)
        c, ck = columns(coords, coord_dtype)
        a, ak = columns(attrs, attr_dtype) if attrs else (None, None)
        arr, keep = grid_specs(grids)
        h = c_void_p()
        check(lib().bin_graph_create_multi(ctypes.byref(c), ctypes.byref(a) if a is not None else None, n, arr,
                                           len(grids), ctypes.byref(h)))
        g._h = h
        g._keep = (c, ck, a, ak, arr, keep)
        return g

    def launch(self, stream=None) -> None:
        check(lib().bin_graph_launch(self._h, _stream_handle(stream)))

    def destroy(self) -> None:
        if self._h:
            check(lib().bin_graph_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def copy_to_host(dev_ptr: int, nbytes: int, dtype, shape):
    """Read nbytes of device memory into a new numpy array."""
    import numpy as np
    a = np.empty(shape, dtype=dtype)
    assert a.nbytes == nbytes
    check(lib().bin_copy_to_host(a.ctypes.data, dev_ptr, nbytes))
    return a


class Server:
    """Continuous-batching request server (binsrv_*).  Column tensors handed
    to submit() are kept referenced until the request is released."""

    def __init__(self, budget_bytes: int = 64 << 30, n_slots: int = 2, max_batch: int = 64, device: int = 0):
        self._h = c_void_p()
        cfg = ServerConfig(budget_bytes, n_slots, max_batch, device, 0)
        check(lib().binsrv_create(ctypes.byref(cfg), ctypes.byref(self._h)))
        self._keep = {}

    def submit(self, coords, attrs, n, axes, bounds, nx, ny, ops, producer_stream=None) -> int:
        """Queue a request; ``producer_stream`` (a torch stream or handle)
        is the stream whose queued work writes the columns, if any."""
        return self.submit_prepared(self.prepare(coords, attrs, n, axes, bounds, nx, ny, ops, producer_stream))

    @staticmethod
    def prepare(coords, attrs, n, axes, bounds, nx, ny, ops, producer_stream=None):
        """A request marshalled once (the arguments of submit), for
        submit_prepared: a caller that submits the same columns every step
        pays the marshalling once."""
        c, ck = columns(coords)
        a, ak = columns(attrs) if attrs else (Columns(None, 0, BIN_F32), None)
        ps = None if producer_stream is None else _stream_handle(producer_stream)
        req = ServerRequest(c, a, n, (c_int32 * 2)(*axes), (c_double * 4)(*bounds), nx, ny, ops, ps)
        return req, (coords, attrs, ck, ak, (nx, ny, ops, len(attrs or [])))

    def submit_prepared(self, prepared) -> int:
        """Queue a request made by prepare()."""
        req, keep = prepared
        t = c_uint64()
        check(lib().binsrv_submit(self._h, ctypes.byref(req), ctypes.byref(t)))
        self._keep[t.value] = keep
        return int(t.value)

    def wait(self, ticket: int, timeout_s: Optional[float] = None) -> Result:
        res = Result()
        ns = -1 if timeout_s is None else int(timeout_s * 1e9)
        check(lib().binsrv_wait(self._h, ticket, ns, ctypes.byref(res)))
        return res

    def fetch(self, ticket: int, res: Result) -> Dict:
        """Copy a finished request's grids to host numpy arrays."""
        import numpy as np
        coords, attrs, _, _, (nx, ny, ops, k) = self._keep[ticket]
        af64 = k > 0 and str(attrs[0].dtype).endswith("float64")
        sa = np.float32 if (not af64 and ops & PREC_PLAIN) else np.float64
        mm = np.float64 if af64 else np.float32
        nb = nx * ny
        out = {}
        if ops & COUNT:
            out["count"] = copy_to_host(res.count, 4 * nb, np.uint32, (ny, nx)).astype(np.int64)
        for key, bit, dt, arr in (("sum", SUM, sa, res.sum), ("min", MIN, mm, res.min), ("max", MAX, mm, res.max),
                                  ("avg", AVG, sa, res.avg)):
            if ops & bit:
                out[key] = [copy_to_host(arr[j], np.dtype(dt).itemsize * nb, dt, (ny, nx)) for j in range(k)]
        return out

    def release(self, ticket: int) -> None:
        check(lib().binsrv_release(self._h, ticket))
        self._keep.pop(ticket, None)

    def stats(self) -> Dict:
        s = ServerStats()
        check(lib().binsrv_get_stats(self._h, ctypes.byref(s)))
        return {n: int(getattr(s, n)) for n, _ in ServerStats._fields_}

    def destroy(self) -> None:
        if self._h:
            check(lib().binsrv_destroy(self._h))
            self._h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def bin_describe_plan(req: Request) -> str:
    buf = ctypes.create_string_buffer(256)
    check(lib().bin_describe_plan(ctypes.byref(req), buf, 256))
    return buf.value.decode()


def bin_describe_plan_on(req: Request, cus: int = 256, lds_per_block: int = 163840, lds_per_cu: int = 163840) -> str:
    """The plan for a device of the given size, without a GPU (MI355X by default)."""
    buf = ctypes.create_string_buffer(512)
    check(lib().bin_describe_plan_on(ctypes.byref(req), cus, lds_per_block, lds_per_cu, buf, 512))
    return buf.value.decode()


def bin_set_plan_override(strategy: int = -1, block: int = 0, grid: int = 0) -> None:
    check(lib().bin_set_plan_override(strategy, block, grid))


TUNE_PART_WG, TUNE_SCATTER_PPT, TUNE_SCATTER_THREADS, TUNE_TILE_SHIFT, TUNE_SPLIT_LEN, TUNE_QUADS = 1, 2, 3, 4, 5, 6


def bin_set_tuning(param: int, value: int) -> None:
    check(lib().bin_set_tuning(param, value))


def reset_tuning() -> None:
    for p in (TUNE_PART_WG, TUNE_SCATTER_PPT, TUNE_SCATTER_THREADS, TUNE_TILE_SHIFT, TUNE_SPLIT_LEN, TUNE_QUADS):
        bin_set_tuning(p, 0)
    bin_set_plan_override(-1, 0, 0)


def bin_timing_enable(on: bool) -> None:
    check(lib().bin_timing_enable(1 if on else 0))


def bin_timing_read():
    """(launches, total_ms) of the dominant kernel since timing was enabled."""
    n = c_int64(0)
    ms = c_double(0)
    check(lib().bin_timing_read(ctypes.byref(n), ctypes.byref(ms)))
    return int(n.value), float(ms.value)


def bin_timing_report() -> Dict[str, tuple]:
    """{kernel name: (launches, total_ms)} since timing was enabled."""
    import json
    buf = ctypes.create_string_buffer(16384)
    check(lib().bin_timing_report(buf, 16384))
    return {k: (int(v[0]), float(v[1])) for k, v in json.loads(buf.value.decode()).items()}


def bin_stream_status(stream=None) -> int:
    return lib().bin_stream_status(_stream_handle(stream))


def bin_release_workspace() -> None:
    check(lib().bin_release_workspace())


def bin_version() -> str:
    return lib().bin_version().decode()
