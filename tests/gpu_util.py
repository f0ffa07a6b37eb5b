"""Helpers for the GPU parity tests (inputs come from the oracle's writer)."""
import os
import sys

import oracle

_CTX = None


def ctx():
    global _CTX
    if _CTX is None:
        from paper_2004_03054_amd import Context
        _CTX = Context(0)
    return _CTX


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def first_diff(a: bytes, b: bytes):
    n = min(len(a), len(b))
    for i in range(n):
        if a[i] != b[i]:
            return i
    return n if len(a) != len(b) else -1


def assert_same_files(gpu_files, ref_files, label=""):
    assert len(gpu_files) == len(ref_files), f"{label}: {len(gpu_files)} files vs oracle {len(ref_files)}"
    for i, (g, r) in enumerate(zip(gpu_files, ref_files)):
        if g != r:
            d = first_diff(g, r)
            raise AssertionError(f"{label}: file {i} differs at byte {d} (sizes {len(g)} vs {len(r)}); "
                                 f"gpu {g[max(0, d - 8):d + 8].hex()} oracle {r[max(0, d - 8):d + 8].hex()}")


def err_tuple(e):
    return (e.status, e.input, e.where, e.phase, e.block, e.offset)
