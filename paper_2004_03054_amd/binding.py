"""ctypes binding of libluda.so (include/luda.h): argument marshalling only.

Every step of a compaction runs in the library's HIP kernels; this module
turns Python buffers into luda_buf arrays and results back into bytes or
device tensors.  It raises if the library is not built.
"""
from __future__ import annotations

import ctypes as C
import os
import struct
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libluda.so")

STATUS = {0: "OK", -1: "INVALID_ARG", -2: "CORRUPT_FORMAT", -3: "CORRUPT_CHECKSUM",
          -4: "UNSORTED_INPUT", -5: "UNSUPPORTED", -6: "NOMEM", -7: "DEVICE", -8: "CANCELLED"}


class LudaBuf(C.Structure):
    _fields_ = [("data", C.c_void_p), ("size", C.c_uint64)]


class LudaOptions(C.Structure):
    _fields_ = [("block_size", C.c_uint32), ("restart_interval", C.c_uint32),
                ("bloom_bits_per_key", C.c_uint32), ("bottommost", C.c_uint32),
                ("target_file_size", C.c_uint64), ("snapshots", C.POINTER(C.c_uint64)),
                ("n_snapshots", C.c_uint32), ("compression", C.c_uint32)]


class LudaError(C.Structure):
    _fields_ = [("status", C.c_int32), ("input", C.c_uint32), ("where", C.c_uint32),
                ("phase", C.c_uint32), ("block", C.c_uint64), ("offset", C.c_uint64)]


class LudaFile(C.Structure):
    _fields_ = [("offset", C.c_uint64), ("size", C.c_uint64), ("num_entries", C.c_uint64),
                ("smallest_off", C.c_uint64), ("smallest_len", C.c_uint64),
                ("largest_off", C.c_uint64), ("largest_len", C.c_uint64)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_void_p, C.c_uint64, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_uint64, C.c_void_p)


class LudaAllocator(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("user", C.c_void_p)]


class LudaResult(C.Structure):
    _fields_ = [("status", C.c_int32), ("error", LudaError), ("num_files", C.c_uint32),
                ("files", C.POINTER(LudaFile)), ("data", C.c_void_p), ("data_size", C.c_uint64),
                ("entries_in", C.c_uint64), ("entries_out", C.c_uint64),
                ("dropped_shadowed", C.c_uint64), ("dropped_tombstones", C.c_uint64),
                ("bytes_in", C.c_uint64), ("bytes_out", C.c_uint64), ("ms_total", C.c_double),
                ("internal", C.c_void_p)]


class LudaJob(C.Structure):
    _fields_ = [("inputs", C.POINTER(LudaBuf)), ("n_inputs", C.c_uint32), ("options", LudaOptions)]


class LudaParams(C.Structure):
    _fields_ = [("crc_waves", C.c_uint32), ("encode_waves", C.c_uint32), ("stride_blocks", C.c_uint32)]


class LudaServerCfg(C.Structure):
    _fields_ = [("hbm_budget", C.c_uint64), ("max_batch_jobs", C.c_uint32), ("workers", C.c_uint32),
                ("host_outputs", C.c_uint32)]


EXPORTS = ["luda_ctx_create", "luda_ctx_destroy", "luda_set_stream", "luda_compact", "luda_compact_dev",
           "luda_compact_batch", "luda_build_tables_dev", "luda_result_free", "luda_status_str",
           "luda_last_error", "luda_stage_times", "luda_selftest_crc", "luda_debug_read", "luda_last_counters",
           "luda_server_create", "luda_server_submit", "luda_server_poll", "luda_server_stats",
           "luda_server_destroy", "luda_get_params", "luda_set_params", "luda_autotune", "luda_set_host_sort",
           "luda_pin_reserve", "luda_pool_trim", "luda_set_allocator", "luda_set_mem_limit", "luda_mem_held",
           "luda_server_cancel", "luda_server_memory"]

_lib = None


def lib():
    """Load libluda.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2004_03054_amd.build_lib.build()")
    # torch first: the library then binds to the HIP runtime torch has
    # loaded, and both share one runtime.  Loaded first, the library would
    # bring in the system runtime, and torch could not initialise its own
    # afterwards.
    import torch  # noqa: F401
    L = C.CDLL(LIB_PATH)
    L.luda_ctx_create.argtypes = [C.c_int, C.POINTER(C.c_void_p)]
    L.luda_ctx_create.restype = C.c_int
    L.luda_ctx_destroy.argtypes = [C.c_void_p]
    L.luda_ctx_destroy.restype = None
    L.luda_set_stream.argtypes = [C.c_void_p, C.c_void_p]
    L.luda_set_stream.restype = C.c_int
    for name in ("luda_compact", "luda_compact_dev"):
        f = getattr(L, name)
        f.argtypes = [C.c_void_p, C.POINTER(LudaBuf), C.c_uint32, C.POINTER(LudaOptions), C.POINTER(LudaResult)]
        f.restype = C.c_int
    L.luda_compact_dev_noalloc.argtypes = [C.c_void_p, C.POINTER(LudaBuf), C.c_uint32, C.POINTER(LudaOptions),
                                           C.c_void_p, C.c_uint64, C.POINTER(LudaResult)]
    L.luda_compact_dev_noalloc.restype = C.c_int
    L.luda_compact_batch.argtypes = [C.c_void_p, C.POINTER(LudaJob), C.c_uint32, C.c_int, C.POINTER(LudaResult)]
    L.luda_compact_batch.restype = C.c_int
    L.luda_build_tables_dev.argtypes = [C.c_void_p, C.c_uint64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                        C.c_void_p, C.POINTER(LudaOptions), C.POINTER(LudaResult)]
    L.luda_build_tables_dev.restype = C.c_int
    L.luda_result_free.argtypes = [C.c_void_p, C.POINTER(LudaResult)]
    L.luda_result_free.restype = None
    L.luda_status_str.argtypes = [C.c_int]
    L.luda_status_str.restype = C.c_char_p
    L.luda_last_error.argtypes = [C.c_void_p]
    L.luda_last_error.restype = C.c_char_p
    L.luda_stage_times.argtypes = [C.c_void_p, C.POINTER(C.c_char_p), C.POINTER(C.c_double), C.c_int]
    L.luda_stage_times.restype = C.c_int
    L.luda_last_counters.argtypes = [C.c_void_p, C.POINTER(C.c_char_p), C.POINTER(C.c_double), C.c_int]
    L.luda_last_counters.restype = C.c_int
    L.luda_debug_read.argtypes = [C.c_void_p, C.c_char_p, C.c_void_p, C.c_uint64, C.c_uint64]
    L.luda_debug_read.restype = C.c_int
    L.luda_selftest_crc.argtypes = []
    L.luda_selftest_crc.restype = C.c_int
    L.luda_get_params.argtypes = [C.c_void_p, C.POINTER(LudaParams)]
    L.luda_get_params.restype = C.c_int
    L.luda_set_params.argtypes = [C.c_void_p, C.POINTER(LudaParams)]
    L.luda_set_params.restype = C.c_int
    L.luda_autotune.argtypes = [C.c_void_p, C.POINTER(LudaJob), C.c_uint32, C.c_int, C.c_uint32,
                                C.POINTER(LudaParams), C.POINTER(C.c_double)]
    L.luda_autotune.restype = C.c_int
    L.luda_server_create.argtypes = [C.c_int, C.POINTER(LudaServerCfg), C.POINTER(C.c_void_p)]
    L.luda_server_create.restype = C.c_int
    L.luda_server_submit.argtypes = [C.c_void_p, C.POINTER(LudaJob), C.POINTER(C.c_uint64)]
    L.luda_server_submit.restype = C.c_int
    L.luda_server_poll.argtypes = [C.c_void_p, C.c_uint64, C.c_int, C.POINTER(LudaResult), C.POINTER(C.c_double)]
    L.luda_server_poll.restype = C.c_int
    L.luda_server_stats.argtypes = [C.c_void_p] + [C.POINTER(C.c_uint64)] * 4
    L.luda_server_stats.restype = C.c_int
    L.luda_set_host_sort.argtypes = [C.c_void_p, C.c_int]
    L.luda_set_host_sort.restype = C.c_int
    L.luda_pin_reserve.argtypes = [C.c_uint64]
    L.luda_pin_reserve.restype = C.c_uint64
    L.luda_pool_trim.argtypes = [C.c_int]
    L.luda_pool_trim.restype = C.c_uint64
    L.luda_server_destroy.argtypes = [C.c_void_p]
    L.luda_server_destroy.restype = None
    L.luda_server_cancel.argtypes = [C.c_void_p, C.c_uint64]
    L.luda_server_cancel.restype = C.c_int
    L.luda_server_memory.argtypes = [C.c_void_p, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)]
    L.luda_server_memory.restype = C.c_int
    L.luda_set_allocator.argtypes = [C.c_void_p, C.POINTER(LudaAllocator)]
    L.luda_set_allocator.restype = C.c_int
    L.luda_set_mem_limit.argtypes = [C.c_void_p, C.c_uint64]
    L.luda_set_mem_limit.restype = C.c_int
    L.luda_mem_held.argtypes = [C.c_void_p]
    L.luda_mem_held.restype = C.c_uint64
    _lib = L
    return L


def options(d: dict) -> LudaOptions:
    """C options from a dict; d["snapshots"] (optional) lists live snapshot
    sequence numbers in ascending order."""
    snaps = [int(x) for x in d.get("snapshots", ())]
    arr = (C.c_uint64 * max(1, len(snaps)))(*snaps)
    o = LudaOptions(int(d["block_size"]), int(d["restart_interval"]), int(d["bloom_bits_per_key"]),
                    int(d["bottommost"]), int(d["target_file_size"]),
                    C.cast(arr, C.POINTER(C.c_uint64)) if snaps else None, len(snaps),
                    int(d.get("compression", 0)))
    o._keep = arr  # the array lives as long as the options
    return o


_JOB_DTYPE = None


def _job_dtype() -> np.dtype:
    """numpy layout of one C job record (offsets taken from the ctypes
    structures, so the two cannot disagree)."""
    global _JOB_DTYPE
    if _JOB_DTYPE is None:
        fields = [("inputs", "<u8", LudaJob.inputs.offset), ("n_inputs", "<u4", LudaJob.n_inputs.offset)]
        base = LudaJob.options.offset
        for name, ct in LudaOptions._fields_:
            fields.append((name, "<u8" if C.sizeof(ct) == 8 else "<u4", base + getattr(LudaOptions, name).offset))
        _JOB_DTYPE = np.dtype({"names": [f[0] for f in fields], "formats": [f[1] for f in fields],
                               "offsets": [f[2] for f in fields], "itemsize": C.sizeof(LudaJob)})
    return _JOB_DTYPE


_OPT_KEYS = ("block_size", "restart_interval", "bloom_bits_per_key", "bottommost", "target_file_size")


def batch_records(jobs: Sequence, device_inputs: bool) -> tuple:
    """The C job records of a batch, (array, keep-alive list): the buffer
    lists of all jobs in one array of (pointer, size) pairs and the records
    filled column by column with numpy, the same bytes options() and one
    buffer list per job would give.  Device inputs are torch tensors, host
    inputs bytes / bytearray / numpy uint8 arrays."""
    J = len(jobs)
    cjobs = (LudaJob * max(1, J))()
    counts = np.fromiter((len(inp) for inp, _ in jobs), dtype=np.int64, count=J)
    n = int(counts.sum())
    flat = np.zeros((max(1, n), 2), dtype=np.uint64)
    keep = [flat]
    if device_inputs:
        ts = [t for inp, _ in jobs for t in inp]
        sizes = [t.numel() for t in ts]
        ptrs = [t.data_ptr() if k else 0 for t, k in zip(ts, sizes)]
    else:
        arrs = []
        for inp, _ in jobs:
            for b in inp:
                a = b if isinstance(b, np.ndarray) else np.frombuffer(bytes(b), dtype=np.uint8)
                arrs.append(np.ascontiguousarray(a, dtype=np.uint8))
        keep.append(arrs)
        sizes = [a.size for a in arrs]
        ptrs = [a.ctypes.data if a.size else 0 for a in arrs]
    if n:
        flat[:, 0] = ptrs
        flat[:, 1] = sizes
    if J:
        rec = np.frombuffer((C.c_uint8 * C.sizeof(cjobs)).from_address(C.addressof(cjobs)), dtype=_job_dtype())
        first = np.concatenate(([0], np.cumsum(counts)[:-1]))
        rec["inputs"][:J] = flat.ctypes.data + 16 * np.minimum(first, max(n - 1, 0)).astype(np.uint64)
        rec["n_inputs"][:J] = counts
        opts = [o for _, o in jobs]
        for k in _OPT_KEYS:
            rec[k][:J] = [int(o[k]) for o in opts]
        rec["compression"][:J] = [int(o.get("compression", 0)) for o in opts]
        for j, o in enumerate(opts):
            snaps = o.get("snapshots", ())
            if len(snaps):
                arr = (C.c_uint64 * len(snaps))(*[int(x) for x in snaps])
                keep.append(arr)
                rec["snapshots"][j] = C.addressof(arr)
                rec["n_snapshots"][j] = len(snaps)
    return cjobs, keep


@dataclass
class Error:
    status: int
    input: int = 0
    where: int = 0
    phase: int = 0
    block: int = 0
    offset: int = 0

    @property
    def name(self) -> str:
        return STATUS.get(self.status, str(self.status))


@dataclass
class Result:
    status: int
    error: Error
    files: list = field(default_factory=list)   # bytes (host) or torch uint8 tensors (device)
    file_entries: List[int] = field(default_factory=list)
    entries_in: int = 0
    entries_out: int = 0
    dropped_shadowed: int = 0
    dropped_tombstones: int = 0
    bytes_in: int = 0
    bytes_out: int = 0
    ms_total: float = 0.0
    file_sizes: List[int] = field(default_factory=list)
    # per file: (smallest key offset, length, largest key offset, length), offsets inside the file
    # (a table whose first data block is stored compressed keeps its smallest key right after it,
    # so that offset is the table's size)
    key_ranges: List[tuple] = field(default_factory=list)
    # per file: (smallest internal key, largest internal key) as bytes, read from the result
    key_bytes: List[tuple] = field(default_factory=list)

    @property
    def name(self) -> str:
        return STATUS.get(self.status, str(self.status))


class _DevView:
    """A __cuda_array_interface__ view of device bytes owned by the library."""

    def __init__(self, ptr: int, n: int):
        self.__cuda_array_interface__ = {"shape": (n,), "typestr": "|u1", "data": (ptr, False),
                                         "version": 2, "strides": None}


def _take(ctx, r: LudaResult, device: bool, materialize: bool = True) -> Result:
    e = r.error
    res = Result(r.status, Error(e.status, e.input, e.where, e.phase, e.block, e.offset),
                 entries_in=r.entries_in, entries_out=r.entries_out, dropped_shadowed=r.dropped_shadowed,
                 dropped_tombstones=r.dropped_tombstones, bytes_in=r.bytes_in, bytes_out=r.bytes_out,
                 ms_total=r.ms_total)
    fs = r.files[:r.num_files] if r.status == 0 and r.num_files else []  # one copy of the file records
    for f in fs:
        res.key_ranges.append((f.smallest_off - f.offset, f.smallest_len, f.largest_off - f.offset, f.largest_len))
        if materialize is not False:
            if device:
                import torch  # device memory plumbing only
                def grab(off, n):
                    return torch.as_tensor(_DevView(r.data + off, n), device="cuda").cpu().numpy().tobytes()
            else:
                def grab(off, n):
                    return C.string_at(r.data + off, n)
            res.key_bytes.append((grab(f.smallest_off, f.smallest_len), grab(f.largest_off, f.largest_len)))
    if r.status == 0 and r.num_files and callable(materialize):
        # apply a function to each output table in place, before the library
        # frees it (no copy): a torch uint8 tensor over device outputs, a
        # numpy uint8 array over host outputs
        for i in range(r.num_files):
            f = r.files[i]
            res.file_entries.append(f.num_entries)
            res.file_sizes.append(f.size)
            if device:
                import torch  # device memory plumbing only
                t = (torch.as_tensor(_DevView(r.data + f.offset, f.size), device="cuda") if f.size
                     else torch.empty(0, dtype=torch.uint8, device="cuda"))
            else:
                t = (np.ctypeslib.as_array((C.c_uint8 * f.size).from_address(r.data + f.offset)) if f.size
                     else np.zeros(0, dtype=np.uint8))
            res.files.append(materialize(t))
    elif r.status == 0 and r.num_files and not materialize:
        res.files = [None] * r.num_files
        res.file_entries = [f.num_entries for f in fs]
        res.file_sizes = [f.size for f in fs]
    elif r.status == 0 and r.num_files:
        import torch  # device memory plumbing only
        for i in range(r.num_files):
            f = r.files[i]
            res.file_entries.append(f.num_entries)
            if device:
                if f.size:
                    t = torch.as_tensor(_DevView(r.data + f.offset, f.size), device="cuda")
                    res.files.append(t.clone())
                else:
                    res.files.append(torch.empty(0, dtype=torch.uint8, device="cuda"))
            else:
                res.files.append(C.string_at(r.data + f.offset, f.size))
    if device and r.status == 0 and r.num_files and materialize:
        # the copies (or the function's reads) were queued on torch's stream:
        # they end before the buffer goes back to the library for reuse
        import torch
        torch.cuda.current_stream().synchronize()
    lib().luda_result_free(ctx, C.byref(r))
    return res


_RES_DTYPE = None


def _np_format(ct) -> str:
    if ct is C.c_double:
        return "<f8"
    if ct is C.c_int32:
        return "<i4"
    return "<u8" if C.sizeof(ct) == 8 else "<u4"


def _res_dtype() -> np.dtype:
    """numpy layout of one C result record, the error record's fields
    flattened as e_<name> (offsets taken from the ctypes structures)."""
    global _RES_DTYPE
    if _RES_DTYPE is None:
        fields = []
        for name, ct in LudaResult._fields_:
            off = getattr(LudaResult, name).offset
            if ct is LudaError:
                for en, et in LudaError._fields_:
                    fields.append(("e_" + en, _np_format(et), off + getattr(LudaError, en).offset))
            else:
                fields.append((name, _np_format(ct), off))
        _RES_DTYPE = np.dtype({"names": [f[0] for f in fields], "formats": [f[1] for f in fields],
                               "offsets": [f[2] for f in fields], "itemsize": C.sizeof(LudaResult)})
    return _RES_DTYPE


_ERR_KEYS = ("e_status", "e_input", "e_where", "e_phase", "e_block", "e_offset")
_RES_KEYS = ("entries_in", "entries_out", "dropped_shadowed", "dropped_tombstones", "bytes_in", "bytes_out",
             "ms_total")


def take_records(res, J: int, free) -> List[Result]:
    """Results of a batch without their output bytes (what _take gives with
    materialize=False): the records' fields read column by column, each
    job's file records unpacked at once; free(res[j]) then hands job j's
    buffers back to the library."""
    if J == 0:
        return []
    rec = np.frombuffer((C.c_uint8 * C.sizeof(res)).from_address(C.addressof(res)), dtype=_res_dtype())[:J]
    col = {n: rec[n].tolist() for n in ("status", "num_files", "files") + _ERR_KEYS + _RES_KEYS}
    errs = zip(*(col[k] for k in _ERR_KEYS))
    vals = zip(*(col[k] for k in _RES_KEYS))  # Result's fields after files and file_entries, in order
    out = []
    for j, (st, nf, fa, e, v) in enumerate(zip(col["status"], col["num_files"], col["files"], errs, vals)):
        r = Result(st, Error(*e), [], [], *v)
        if st == 0 and nf:
            n7 = 7 * nf  # a file record is seven uint64 fields
            w = struct.unpack_from("<%dQ" % n7, C.string_at(fa, 8 * n7))
            r.key_ranges = [(w[i + 3] - w[i], w[i + 4], w[i + 5] - w[i], w[i + 6]) for i in range(0, n7, 7)]
            r.files = [None] * nf
            r.file_entries = list(w[2::7])
            r.file_sizes = list(w[1::7])
        free(res[j])
        out.append(r)
    return out


def _bufs(inputs) -> tuple:
    """Host inputs: bytes / bytearray / numpy uint8 arrays (kept alive by the caller)."""
    arrs = []
    bufs = (LudaBuf * max(1, len(inputs)))()
    for i, b in enumerate(inputs):
        a = b if isinstance(b, np.ndarray) else np.frombuffer(bytes(b), dtype=np.uint8)
        a = np.ascontiguousarray(a, dtype=np.uint8)
        arrs.append(a)
        bufs[i].data = a.ctypes.data if a.size else None
        bufs[i].size = a.size
    return bufs, arrs


def _torch_sync():
    """Device inputs written on torch's current stream must be complete before
    the library's own (non-blocking) streams read them.  Only that stream is
    waited for: a device-wide synchronize would also wait for the passes the
    library's other contexts and server workers have in flight.  Inputs
    written on other torch streams are the caller's to order."""
    import torch
    torch.cuda.current_stream().synchronize()


def _dev_bufs(inputs, sync: bool = True) -> LudaBuf:
    if sync:
        _torch_sync()
    bufs = (LudaBuf * max(1, len(inputs)))()
    for i, t in enumerate(inputs):
        bufs[i].data = t.data_ptr() if t.numel() else None
        bufs[i].size = t.numel()
    return bufs


class Context:
    """A library context on one HIP device."""

    def __init__(self, device: int = 0):
        self._h = C.c_void_p()
        self._alloc = None
        rc = lib().luda_ctx_create(device, C.byref(self._h))
        if rc != 0:
            raise RuntimeError(f"luda_ctx_create failed: {STATUS.get(rc, rc)}")

    def close(self):
        if self._h:
            lib().luda_ctx_destroy(self._h)
            self._h = C.c_void_p()
            self._alloc = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_stream(self, stream_handle: Optional[int]):
        lib().luda_set_stream(self._h, C.c_void_p(stream_handle) if stream_handle else None)

    def last_error(self) -> str:
        return lib().luda_last_error(self._h).decode()

    def compact(self, inputs: Sequence, opts: dict, materialize: bool = True) -> Result:
        """Host tables in, host tables out.  With materialize=False the
        output tables are released unread (sizes only)."""
        bufs, _keep = _bufs(inputs)
        o = options(opts)
        r = LudaResult()
        lib().luda_compact(self._h, bufs, len(inputs), C.byref(o), C.byref(r))
        return _take(self._h, r, device=False, materialize=materialize)

    def compact_dev(self, inputs: Sequence, opts: dict, materialize: bool = True) -> Result:
        """Device (torch uint8 cuda tensors) tables in, device tensors out.
        With materialize=False the output tables are released unread (sizes only)."""
        bufs = _dev_bufs(inputs)
        o = options(opts)
        r = LudaResult()
        lib().luda_compact_dev(self._h, bufs, len(inputs), C.byref(o), C.byref(r))
        return _take(self._h, r, device=True, materialize=materialize)

    def compact_dev_noalloc(self, inputs: Sequence, opts: dict, out, materialize: bool = True) -> Result:
        """compact_dev without device allocations: working buffers in the
        library's static scratch memory, output tables written into `out` (a
        torch uint8 cuda tensor).  The returned tables view `out` unless
        materialize is a function (e.g. a clone) or False."""
        bufs = _dev_bufs(inputs)
        o = options(opts)
        r = LudaResult()
        lib().luda_compact_dev_noalloc(self._h, bufs, len(inputs), C.byref(o),
                                       C.c_void_p(out.data_ptr() if out.numel() else None), out.numel(), C.byref(r))
        return _take(self._h, r, device=True, materialize=materialize if materialize is not True else (lambda t: t))

    def compact_batch(self, jobs: Sequence, device_inputs: bool, materialize: bool = True) -> List[Result]:
        """jobs: sequence of (inputs, options dict)."""
        J = len(jobs)
        cjobs, _keep = self._jobs(jobs, device_inputs)
        res = (LudaResult * max(1, J))()
        rc = lib().luda_compact_batch(self._h, cjobs, J, 1 if device_inputs else 0, res)
        if materialize is False:
            out = take_records(res, J, lambda r: lib().luda_result_free(self._h, C.byref(r)))
        else:
            out = [_take(self._h, res[j], device=device_inputs, materialize=materialize) for j in range(J)]
        if rc != 0 and J:
            for o in out:
                if o.status == 0:
                    o.status = rc
        return out

    def _jobs(self, jobs: Sequence, device_inputs: bool):
        if device_inputs:
            _torch_sync()  # once for the whole batch
        return batch_records(jobs, device_inputs)

    def set_mem_limit(self, nbytes: int):
        """Most device bytes the context's buffers may hold at once (0: none)."""
        lib().luda_set_mem_limit(self._h, int(nbytes))

    def mem_held(self) -> int:
        return int(lib().luda_mem_held(self._h))

    def use_torch_allocator(self, on: bool = True):
        """Take the context's device memory from PyTorch's caching allocator
        (luda_set_allocator), or (on=False) from hipMalloc again."""
        if not on:
            rc = lib().luda_set_allocator(self._h, None)
            self._alloc = None
            if rc != 0:
                raise RuntimeError(f"luda_set_allocator: {STATUS.get(rc, rc)}")
            return
        import torch  # device memory plumbing only
        dev = torch.cuda.current_device()

        def _alloc(user, nbytes, stream):
            try:
                return torch.cuda.caching_allocator_alloc(int(nbytes), dev, int(stream or 0))
            except Exception:  # noqa: BLE001 - out of memory is reported as NULL
                return None

        def _free(user, ptr, nbytes, stream):
            torch.cuda.caching_allocator_delete(int(ptr))

        a = LudaAllocator(ALLOC_FN(_alloc), FREE_FN(_free), None)
        rc = lib().luda_set_allocator(self._h, C.byref(a))
        if rc != 0:
            raise RuntimeError(f"luda_set_allocator: {STATUS.get(rc, rc)}")
        self._alloc = a  # the callbacks live as long as the context uses them

    def set_host_sort(self, on: bool):
        """Cooperative sort: order the entries on the host instead of merging
        them on the device (same output bytes)."""
        rc = lib().luda_set_host_sort(self._h, 1 if on else 0)
        if rc != 0:
            raise ValueError(f"luda_set_host_sort: {STATUS.get(rc, rc)}")

    def params(self) -> dict:
        p = LudaParams()
        lib().luda_get_params(self._h, C.byref(p))
        return dict(crc_waves=p.crc_waves, encode_waves=p.encode_waves, stride_blocks=p.stride_blocks)

    def set_params(self, crc_waves: int, encode_waves: int, stride_blocks: int):
        rc = lib().luda_set_params(self._h, C.byref(LudaParams(crc_waves, encode_waves, stride_blocks)))
        if rc != 0:
            raise ValueError(f"luda_set_params: {STATUS.get(rc, rc)}")

    def autotune(self, jobs: Sequence, device_inputs: bool, rounds: int = 2) -> tuple:
        """(best params dict, best ms) over the given jobs; the context keeps them."""
        cjobs, _keep = self._jobs(jobs, device_inputs)
        p = LudaParams()
        ms = C.c_double()
        rc = lib().luda_autotune(self._h, cjobs, len(jobs), 1 if device_inputs else 0, rounds, C.byref(p),
                                 C.byref(ms))
        if rc != 0:
            raise RuntimeError(f"luda_autotune: {STATUS.get(rc, rc)} {self.last_error()}")
        return dict(crc_waves=p.crc_waves, encode_waves=p.encode_waves, stride_blocks=p.stride_blocks), ms.value

    def build_tables_dev(self, keys, koff, tags, vals, voff, opts: dict) -> Result:
        """Write ordered entries (device tensors) into tables on the device."""
        o = options(opts)
        r = LudaResult()
        n = tags.numel()
        _torch_sync()
        lib().luda_build_tables_dev(self._h, n, keys.data_ptr(), koff.data_ptr(), tags.data_ptr(),
                                    vals.data_ptr(), voff.data_ptr(), C.byref(o), C.byref(r))
        return _take(self._h, r, device=True)

    def debug_read(self, name: str, dtype, count: int, offset: int = 0) -> np.ndarray:
        """Copy `count` elements of an internal device buffer of the last call."""
        a = np.zeros(count, dtype=dtype)
        rc = lib().luda_debug_read(self._h, name.encode(), a.ctypes.data, offset * a.itemsize, a.nbytes)
        if rc != 0:
            raise RuntimeError(f"debug_read({name}) failed: {STATUS.get(rc, rc)}")
        return a

    def stage_times(self) -> List[tuple]:
        names = (C.c_char_p * 64)()
        ms = (C.c_double * 64)()
        n = lib().luda_stage_times(self._h, names, ms, 64)
        return [(names[i].decode(), ms[i]) for i in range(min(n, 64))]

    def counters(self) -> dict:
        names = (C.c_char_p * 64)()
        vals = (C.c_double * 64)()
        n = lib().luda_last_counters(self._h, names, vals, 64)
        return {names[i].decode(): vals[i] for i in range(min(n, 64))}


def selftest_crc() -> int:
    return lib().luda_selftest_crc()


def pool_trim(device: int = 0) -> int:
    """Free the device's pooled output buffers (luda_pool_trim); returns the
    bytes freed."""
    return int(lib().luda_pool_trim(int(device)))


def pin_reserve(nbytes: int) -> int:
    """Pin host memory ahead of time for results in host memory (see
    luda_pin_reserve); returns the pinned pool's size in bytes."""
    return int(lib().luda_pin_reserve(int(nbytes)))


class Server:
    """The served form: jobs with device inputs are submitted as they arrive
    and collected by ticket (luda_server_* of include/luda.h)."""

    def __init__(self, device: int = 0, hbm_budget: int = 64 << 30, max_batch_jobs: int = 0, workers: int = 2,
                 host_outputs: bool = True):
        self._h = C.c_void_p()
        cfg = LudaServerCfg(hbm_budget, max_batch_jobs, workers, 1 if host_outputs else 0)
        rc = lib().luda_server_create(device, C.byref(cfg), C.byref(self._h))
        if rc != 0:
            raise RuntimeError(f"luda_server_create failed: {STATUS.get(rc, rc)}")
        self._host = host_outputs
        self._keep = {}

    def submit(self, inputs: Sequence, opts: dict) -> int:
        """inputs: torch uint8 cuda tensors (kept alive until collected)."""
        bufs = _dev_bufs(inputs)
        job = LudaJob()
        job.inputs = C.cast(bufs, C.POINTER(LudaBuf))
        job.n_inputs = len(inputs)
        o = options(opts)  # its snapshot array is copied by the submit
        job.options = o
        t = C.c_uint64()
        rc = lib().luda_server_submit(self._h, C.byref(job), C.byref(t))
        if rc == -6:
            raise MemoryError("luda_server_submit: the job's expected footprint exceeds the HBM budget")
        if rc != 0:
            raise RuntimeError(f"luda_server_submit failed: {STATUS.get(rc, rc)}")
        self._keep[t.value] = (bufs, list(inputs))
        return t.value

    def poll(self, ticket: int, wait: bool = True, materialize=True):
        """(Result, latency_ms), or None if not complete (wait=False)."""
        r = LudaResult()
        lat = C.c_double()
        rc = lib().luda_server_poll(self._h, ticket, 1 if wait else 0, C.byref(r), C.byref(lat))
        if rc == 1:
            return None
        if rc != 0:
            raise RuntimeError(f"luda_server_poll failed: {STATUS.get(rc, rc)}")
        self._keep.pop(ticket, None)
        return _take(None, r, device=not self._host, materialize=materialize), lat.value

    def cancel(self, ticket: int) -> bool:
        """Withdraw a job no worker has taken yet (True), else False."""
        rc = lib().luda_server_cancel(self._h, ticket)
        if rc < 0:
            raise RuntimeError(f"luda_server_cancel failed: {STATUS.get(rc, rc)}")
        return rc == 0

    def memory(self) -> dict:
        h, u = C.c_uint64(), C.c_uint64()
        lib().luda_server_memory(self._h, C.byref(h), C.byref(u))
        return dict(held_by_workers=h.value, device_used=u.value)

    def stats(self) -> dict:
        v = [C.c_uint64() for _ in range(4)]
        lib().luda_server_stats(self._h, *[C.byref(x) for x in v])
        return dict(jobs=v[0].value, batches=v[1].value, max_batch=v[2].value, peak_admitted=v[3].value)

    def close(self):
        if self._h:
            lib().luda_server_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
