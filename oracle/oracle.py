"""ctypes binding of the oracle library (test infrastructure only)."""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "luda_oracle.c")
_LIB = os.path.join(_HERE, "libluda_oracle.so")

STATUS_NAMES = {0: "OK", -1: "INVALID_ARG", -2: "CORRUPT_FORMAT", -3: "CORRUPT_CHECKSUM",
                -4: "UNSORTED_INPUT", -5: "UNSUPPORTED", -6: "NOMEM"}
STATUS_CODES = {v: k for k, v in STATUS_NAMES.items()}
WHERE_NAMES = {0: "footer", 1: "index", 2: "data"}
PHASE_NAMES = {0: "trailer", 1: "restarts", 2: "entries"}


_SAN_LIB = os.path.join(_HERE, "libluda_oracle_san.so")


def build(force: bool = True, sanitize: bool = False) -> str:
    """Compile the oracle with gcc into oracle/libluda_oracle.so; with
    sanitize, an AddressSanitizer + UndefinedBehaviorSanitizer build into
    oracle/libluda_oracle_san.so (loaded when LUDA_ORACLE_SANITIZE=1, with
    libasan preloaded into the interpreter)."""
    lib_path = _SAN_LIB if sanitize else _LIB
    if force or not os.path.exists(lib_path):
        tmp = lib_path + ".tmp"
        flags = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                 "-fno-sanitize-recover=undefined"] if sanitize else ["-O2"]
        subprocess.check_call(["gcc"] + flags + ["-std=gnu11", "-Wall", "-shared", "-fPIC", "-o", tmp, _SRC])
        os.replace(tmp, lib_path)
    return lib_path


class _Options(C.Structure):
    _fields_ = [("block_size", C.c_uint32), ("restart_interval", C.c_uint32),
                ("bloom_bits_per_key", C.c_uint32), ("bottommost", C.c_uint32),
                ("target_file_size", C.c_uint64), ("snapshots", C.POINTER(C.c_uint64)),
                ("n_snapshots", C.c_uint32), ("compression", C.c_uint32)]


class _Error(C.Structure):
    _fields_ = [("status", C.c_int32), ("input", C.c_uint32), ("where", C.c_uint32),
                ("phase", C.c_uint32), ("block", C.c_uint64), ("offset", C.c_uint64)]


class _Entries(C.Structure):
    _fields_ = [("n", C.c_uint64), ("keys", C.c_void_p), ("koff", C.c_void_p),
                ("tags", C.c_void_p), ("vals", C.c_void_p), ("voff", C.c_void_p)]


class _Decoded(C.Structure):
    _fields_ = [("n", C.c_uint64), ("keys", C.POINTER(C.c_uint8)), ("koff", C.POINTER(C.c_uint64)),
                ("tags", C.POINTER(C.c_uint64)), ("vals", C.POINTER(C.c_uint8)),
                ("voff", C.POINTER(C.c_uint64))]


class _Result(C.Structure):
    _fields_ = [("num_files", C.c_uint32), ("file_off", C.POINTER(C.c_uint64)),
                ("data", C.POINTER(C.c_uint8)),
                ("entries_in", C.c_uint64), ("entries_out", C.c_uint64),
                ("dropped_shadowed", C.c_uint64), ("dropped_tombstones", C.c_uint64),
                ("bytes_in", C.c_uint64), ("bytes_out", C.c_uint64),
                ("n_inputs", C.c_uint32), ("input_first", C.POINTER(C.c_uint64)),
                ("surv", C.POINTER(C.c_uint64)), ("n_blocks", C.c_uint64),
                ("block_first", C.POINTER(C.c_uint64)),
                ("file_first_block", C.POINTER(C.c_uint64))]


_lib = None


def lib():
    global _lib
    if _lib is None:
        san = os.environ.get("LUDA_ORACLE_SANITIZE") == "1"
        path = build(force=False, sanitize=san)
        L = C.CDLL(path)
        u8p, u64 = C.c_void_p, C.c_uint64
        L.ref_crc32c.argtypes = [u8p, u64]; L.ref_crc32c.restype = C.c_uint32
        L.ref_crc32c_bitwise.argtypes = [u8p, u64]; L.ref_crc32c_bitwise.restype = C.c_uint32
        L.ref_crc32c_extend.argtypes = [C.c_uint32, u8p, u64]; L.ref_crc32c_extend.restype = C.c_uint32
        L.ref_mask_crc.argtypes = [C.c_uint32]; L.ref_mask_crc.restype = C.c_uint32
        L.ref_unmask_crc.argtypes = [C.c_uint32]; L.ref_unmask_crc.restype = C.c_uint32
        L.ref_xxh64.argtypes = [u8p, u64, u64]; L.ref_xxh64.restype = C.c_uint64
        L.ref_put_varint64.argtypes = [u8p, u64]; L.ref_put_varint64.restype = C.c_int
        L.ref_get_varint32.argtypes = [u8p, u8p, C.POINTER(C.c_uint32)]; L.ref_get_varint32.restype = C.c_int
        L.ref_get_varint64.argtypes = [u8p, u8p, C.POINTER(C.c_uint64)]; L.ref_get_varint64.restype = C.c_int
        L.ref_bloom_size.argtypes = [u64, C.c_uint32]; L.ref_bloom_size.restype = C.c_uint64
        L.ref_bloom_build.argtypes = [u8p, u8p, u64, C.c_uint32, u8p]; L.ref_bloom_build.restype = None
        L.ref_bloom_may_match.argtypes = [u8p, u64, u8p, u64]; L.ref_bloom_may_match.restype = C.c_int
        L.ref_build_tables.argtypes = [C.POINTER(_Entries), C.POINTER(_Options), C.POINTER(C.POINTER(_Result))]
        L.ref_build_tables.restype = C.c_int
        L.ref_decode_table.argtypes = [u8p, u64, C.c_uint32, C.POINTER(C.POINTER(_Decoded)), C.POINTER(_Error)]
        L.ref_decode_table.restype = C.c_int
        L.ref_compact.argtypes = [C.POINTER(C.c_void_p), C.POINTER(C.c_uint64), C.c_uint32,
                                  C.POINTER(_Options), C.POINTER(C.POINTER(_Result)), C.POINTER(_Error)]
        L.ref_compact.restype = C.c_int
        L.ref_snappy_decompress.argtypes = [u8p, u64, C.POINTER(C.POINTER(C.c_uint8)), C.POINTER(C.c_uint64),
                                            C.POINTER(C.c_uint64)]
        L.ref_snappy_decompress.restype = C.c_int
        L.ref_snappy_max.argtypes = [u64]; L.ref_snappy_max.restype = C.c_uint64
        L.ref_snappy_compress.argtypes = [u8p, u64, u8p]; L.ref_snappy_compress.restype = C.c_uint64
        L.free.argtypes = [C.c_void_p]; L.free.restype = None
        L.ref_free_result.argtypes = [C.POINTER(_Result)]; L.ref_free_result.restype = None
        L.ref_free_decoded.argtypes = [C.POINTER(_Decoded)]; L.ref_free_decoded.restype = None
        _lib = L
    return _lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data if a.size else 0


def _u8(b) -> np.ndarray:
    if isinstance(b, np.ndarray):
        return np.ascontiguousarray(b, dtype=np.uint8)
    return np.frombuffer(bytes(b), dtype=np.uint8)


def crc32c(b) -> int:
    a = _u8(b)
    return lib().ref_crc32c(_ptr(a), a.size)


def crc32c_bitwise(b) -> int:
    a = _u8(b)
    return lib().ref_crc32c_bitwise(_ptr(a), a.size)


def crc32c_extend(crc: int, b) -> int:
    a = _u8(b)
    return lib().ref_crc32c_extend(crc, _ptr(a), a.size)


def mask_crc(c: int) -> int:
    return lib().ref_mask_crc(c)


def unmask_crc(c: int) -> int:
    return lib().ref_unmask_crc(c)


def xxh64(b, seed: int = 0) -> int:
    a = _u8(b)
    return lib().ref_xxh64(_ptr(a), a.size, seed)


def put_varint64(v: int) -> bytes:
    buf = np.zeros(16, np.uint8)
    n = lib().ref_put_varint64(_ptr(buf), v)
    return buf[:n].tobytes()


def get_varint32(b):
    a = _u8(b) if len(b) else np.zeros(1, np.uint8)
    v = C.c_uint32()
    n = lib().ref_get_varint32(_ptr(a), _ptr(a) + len(b), C.byref(v))
    return (v.value, n) if n else (None, 0)


def get_varint64(b):
    a = _u8(b) if len(b) else np.zeros(1, np.uint8)
    v = C.c_uint64()
    n = lib().ref_get_varint64(_ptr(a), _ptr(a) + len(b), C.byref(v))
    return (v.value, n) if n else (None, 0)


def bloom_size(n: int, bits_per_key: int = 10) -> int:
    return lib().ref_bloom_size(n, bits_per_key)


def bloom_build(keys: Sequence[bytes], bits_per_key: int = 10) -> bytes:
    data = _u8(b"".join(keys)) if keys else np.zeros(1, np.uint8)
    koff = np.zeros(len(keys) + 1, np.uint64)
    koff[1:] = np.cumsum([len(k) for k in keys]) if keys else []
    out = np.zeros(bloom_size(len(keys), bits_per_key), np.uint8)
    lib().ref_bloom_build(_ptr(data), _ptr(koff), len(keys), bits_per_key, _ptr(out))
    return out.tobytes()


def bloom_may_match(filt: bytes, key: bytes) -> bool:
    f = _u8(filt)
    k = _u8(key) if key else np.zeros(1, np.uint8)
    return bool(lib().ref_bloom_may_match(_ptr(f), f.size, _ptr(k), len(key)))


def snappy_compress(b) -> bytes:
    """The writer's Snappy stream for a block's raw bytes."""
    a = _u8(b) if len(b) else np.zeros(1, np.uint8)
    out = np.zeros(lib().ref_snappy_max(len(b)), dtype=np.uint8)
    n = lib().ref_snappy_compress(_ptr(a), len(b), _ptr(out))
    return out[:n].tobytes()


def snappy_decompress(b):
    """(status, bytes or None, error offset) for a Snappy stream."""
    a = _u8(b) if len(b) else np.zeros(1, np.uint8)
    p = C.POINTER(C.c_uint8)()
    n = C.c_uint64()
    at = C.c_uint64()
    st = lib().ref_snappy_decompress(_ptr(a), len(b), C.byref(p), C.byref(n), C.byref(at))
    if st != 0:
        return st, None, at.value
    out = bytes(C.string_at(p, n.value)) if n.value else b""
    lib().free(C.cast(p, C.c_void_p))
    return st, out, 0


def _opts(o: dict) -> _Options:
    """Options for the C oracle; o["snapshots"] (optional) lists the live
    snapshot sequence numbers in ascending order."""
    snaps = [int(x) for x in o.get("snapshots", ())]
    arr = (C.c_uint64 * max(1, len(snaps)))(*snaps)
    r = _Options(int(o["block_size"]), int(o["restart_interval"]), int(o["bloom_bits_per_key"]),
                 int(o["bottommost"]), int(o["target_file_size"]), C.cast(arr, C.POINTER(C.c_uint64)),
                 len(snaps), int(o.get("compression", 0)))
    r._keep = arr  # the array lives as long as the options
    return r


@dataclass
class RefError:
    status: int
    input: int = 0
    where: int = 0
    phase: int = 0
    block: int = 0
    offset: int = 0

    @property
    def name(self) -> str:
        return STATUS_NAMES.get(self.status, str(self.status))

    def __str__(self):
        return (f"{self.name}: input {self.input} {WHERE_NAMES.get(self.where)} block {self.block} "
                f"{PHASE_NAMES.get(self.phase)} @ {self.offset}")


@dataclass
class RefResult:
    status: int
    error: RefError
    files: List[bytes] = field(default_factory=list)
    entries_in: int = 0
    entries_out: int = 0
    dropped_shadowed: int = 0
    dropped_tombstones: int = 0
    bytes_in: int = 0
    bytes_out: int = 0
    input_first: Optional[np.ndarray] = None
    surv: Optional[np.ndarray] = None
    block_first: Optional[np.ndarray] = None
    file_first_block: Optional[np.ndarray] = None


def _arr(p, n, dtype=np.uint64) -> np.ndarray:
    if n == 0 or not p:
        return np.zeros(0, dtype)
    return np.ctypeslib.as_array(p, shape=(n,)).astype(dtype, copy=True)


def _take_result(rp, status: int, err: RefError) -> RefResult:
    r = rp.contents
    nf = r.num_files
    fo = _arr(r.file_off, nf + 1)
    total = int(fo[-1]) if nf else 0
    data = bytes(C.string_at(r.data, total)) if total else b""
    files = [data[int(fo[i]):int(fo[i + 1])] for i in range(nf)]
    out = RefResult(status, err, files, r.entries_in, r.entries_out, r.dropped_shadowed,
                    r.dropped_tombstones, r.bytes_in, r.bytes_out,
                    _arr(r.input_first, r.n_inputs + 1) if r.input_first else None,
                    _arr(r.surv, r.entries_out) if r.surv else None,
                    _arr(r.block_first, r.n_blocks + 1), _arr(r.file_first_block, nf + 1))
    lib().ref_free_result(rp)
    return out


def build_tables(keys: np.ndarray, koff: np.ndarray, tags: np.ndarray, vals: np.ndarray,
                 voff: np.ndarray, options: dict) -> RefResult:
    """Phase 3 over an ordered entry list (already deduplicated)."""
    keys = _u8(keys) if keys.size else np.zeros(1, np.uint8)
    vals = _u8(vals) if vals.size else np.zeros(1, np.uint8)
    koff = np.ascontiguousarray(koff, np.uint64)
    voff = np.ascontiguousarray(voff, np.uint64)
    tags = np.ascontiguousarray(tags, np.uint64)
    ent = _Entries(tags.size, _ptr(keys), _ptr(koff), _ptr(tags), _ptr(vals), _ptr(voff))
    o = _opts(options)
    rp = C.POINTER(_Result)()
    st = lib().ref_build_tables(C.byref(ent), C.byref(o), C.byref(rp))
    if st != 0:
        return RefResult(st, RefError(st))
    return _take_result(rp, st, RefError(0))


def build_input_tables(job) -> List[bytes]:
    """Write each run of a workload job as one input table (oracle writer)."""
    out = []
    for r in job.runs:
        res = build_tables(r.keys, r.koff, r.tags, r.vals, r.voff, job.table_options())
        if res.status != 0:
            raise RuntimeError(f"oracle table writer failed: {res.error}")
        assert len(res.files) <= 1
        out.append(res.files[0] if res.files else b"")
    return out


def decode_table(sst: bytes, input_index: int = 0):
    """Phase 1 for one table -> (status, RefError, (keys list, tags array, values list))."""
    a = _u8(sst) if len(sst) else np.zeros(1, np.uint8)
    dp = C.POINTER(_Decoded)()
    e = _Error()
    st = lib().ref_decode_table(_ptr(a), len(sst), input_index, C.byref(dp), C.byref(e))
    err = RefError(e.status, e.input, e.where, e.phase, e.block, e.offset)
    if st != 0:
        return st, err, None
    d = dp.contents
    n = d.n
    koff = _arr(d.koff, n + 1)
    voff = _arr(d.voff, n + 1)
    keys = bytes(C.string_at(d.keys, int(koff[-1]))) if n and koff[-1] else b""
    vals = bytes(C.string_at(d.vals, int(voff[-1]))) if n and voff[-1] else b""
    tags = _arr(d.tags, n)
    lib().ref_free_decoded(dp)
    return st, err, ([keys[koff[i]:koff[i + 1]] for i in range(n)], tags,
                     [vals[voff[i]:voff[i + 1]] for i in range(n)])


def compact(inputs: Sequence[bytes], options: dict) -> RefResult:
    """The whole job; inputs[0] is the upper (newest) table."""
    arrs = [_u8(b) if len(b) else np.zeros(1, np.uint8) for b in inputs]
    ptrs = (C.c_void_p * max(1, len(arrs)))(*[_ptr(a) for a in arrs])
    sizes = (C.c_uint64 * max(1, len(arrs)))(*[len(b) for b in inputs])
    o = _opts(options)
    rp = C.POINTER(_Result)()
    e = _Error()
    st = lib().ref_compact(ptrs, sizes, len(inputs), C.byref(o), C.byref(rp), C.byref(e))
    err = RefError(e.status, e.input, e.where, e.phase, e.block, e.offset)
    if st != 0:
        return RefResult(st, err)
    return _take_result(rp, st, err)


def compact_job(job, inputs: Optional[List[bytes]] = None) -> RefResult:
    if inputs is None:
        inputs = build_input_tables(job)
    return compact(inputs, job.options())
