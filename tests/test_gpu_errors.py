"""GPU error parity: the same status and first-corruption location as the
oracle, for corruptions planted on the host."""
import struct

import numpy as np
import pytest

import oracle
from gpu_util import ctx, err_tuple, say
from test_oracle_errors import _tables, handles, reseal
from sstcheck import varint

pytestmark = pytest.mark.gpu


def both(tables, opts, label):
    say(f"[gpu] errors: {label}")
    ins = [bytes(t) for t in tables]
    ref = oracle.compact(ins, opts)
    res = ctx().compact(ins, opts)
    assert res.status == ref.status, (label, res.name, ref.error, ctx().last_error())
    if ref.status:
        assert err_tuple(res.error) == err_tuple(ref.error), (label, res.error, ref.error)
        assert res.files == []


def test_clean():
    job, ts = _tables()
    both(ts, job.options(), "clean")


def test_checksum_and_precedence():
    job, ts = _tables()
    _, hs = handles(ts[1])
    bo, bs = hs[len(hs) // 2]
    ts[1][bo + bs // 2] ^= 0x40
    both(ts, job.options(), "checksum")
    job, ts = _tables()
    _, h0 = handles(ts[0])
    _, h2 = handles(ts[2])
    ts[2][h2[0][0]] ^= 1
    ts[0][h0[-1][0]] ^= 1
    both(ts, job.options(), "two inputs")
    job, ts = _tables(seed=2)
    _, h1 = handles(ts[1])
    ts[1][h1[2][0]] ^= 1
    ts[1][h1[1][0]] ^= 1
    both(ts, job.options(), "two blocks")


def test_footer_and_index():
    job, ts = _tables()
    t = bytes(ts[0])
    both([t[:-1]] + [bytes(x) for x in ts[1:]], job.options(), "truncated")
    both([bytes(x) for x in ts[:2]] + [b"\x00" * 20], job.options(), "short")
    bad = bytearray(t)
    bad[-1] ^= 0xFF
    both([bad], job.options(), "magic")
    (io, isz), hs = handles(ts[1])
    x = bytearray(ts[1])
    x[io + 1] ^= 0x10
    both([ts[0], x], job.options(), "index crc")


def test_block_level_errors():
    job, ts = _tables()
    _, hs = handles(ts[0])
    bo, bs = hs[0]
    t = bytearray(ts[0])
    t[bo + bs] = 1
    reseal(t, bo, bs)
    both([t], job.options(), "raw contents marked compressed")
    t = bytearray(ts[0])
    t[bo + bs] = 2
    reseal(t, bo, bs)
    both([t], job.options(), "unknown block type")
    nr = struct.unpack_from("<I", ts[0], bo + bs - 4)[0]
    t = bytearray(ts[0])
    t[bo + bs - 4:bo + bs] = struct.pack("<I", bs)
    reseal(t, bo, bs)
    both([t], job.options(), "restart count")
    t = bytearray(ts[0])
    de = bs - 4 - 4 * nr
    t[bo + de:bo + de + 4] = struct.pack("<I", 1)
    reseal(t, bo, bs)
    both([t], job.options(), "restart zero")
    t = bytearray(ts[0])
    t[bo] = 1
    reseal(t, bo, bs)
    both([t], job.options(), "shared at restart")
    t = bytearray(ts[0])
    s, q = varint(t, bo, bo + bs, 5)
    ns, q = varint(t, q, bo + bs, 5)
    vl, q = varint(t, q, bo + bs, 5)
    t[q + ns - 8] = 7
    reseal(t, bo, bs)
    both([t], job.options(), "bad type")


def test_unsorted():
    opts = dict(block_size=4096, restart_interval=16, bloom_bits_per_key=10, bottommost=0,
                target_file_size=1 << 40)
    tags = np.array([(5 << 8) | 1] * 3, np.uint64)
    res = oracle.build_tables(np.frombuffer(b"bac", np.uint8), np.array([0, 1, 2, 3], np.uint64), tags,
                              np.zeros(0, np.uint8), np.zeros(4, np.uint64), opts)
    both([res.files[0]], opts, "unsorted")
    res = oracle.build_tables(np.frombuffer(b"aa", np.uint8), np.array([0, 1, 2], np.uint64), tags[:2],
                              np.zeros(0, np.uint8), np.zeros(3, np.uint64), opts)
    both([res.files[0]], opts, "equal keys")
