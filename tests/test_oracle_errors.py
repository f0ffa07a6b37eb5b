"""Error detection and precedence of the oracle, on corruptions made here.

Every corruption is planted on the host into table bytes; the expected status
and location follow from the reading order (footer, index block, data blocks
in index order; inside a block: trailer, restart array, entries in order).
"""
import struct

import numpy as np
import pytest

import oracle
from sstcheck import crc32c_bitwise, enc_varint, mask, varint
from workload import tiny_job

NAMES = {v: k for k, v in oracle.STATUS_NAMES.items()}


def _tables(seed=1, **kw):
    job = tiny_job(seed, n_inputs=3, entries=60, key_alphabet=4, key_len=(2, 4), val_len=(0, 30),
                   p_tomb=0.2, mode="leveled", block_size=128, restart_interval=3, **kw)
    return job, [bytearray(t) for t in oracle.build_input_tables(job)]


def handles(t: bytes):
    ft = t[-48:-8]
    _, p = varint(ft, 0, 40)
    _, p = varint(ft, p, 40)
    ioff, p = varint(ft, p, 40)
    isize, p = varint(ft, p, 40)
    c = t[ioff:ioff + isize]
    nr = struct.unpack_from("<I", c, len(c) - 4)[0]
    de = len(c) - 4 - 4 * nr
    out = []
    o = 0
    while o < de:
        s, q = varint(c, o, de, 5)
        ns, q = varint(c, q, de, 5)
        vl, q = varint(c, q, de, 5)
        v = c[q + ns:q + ns + vl]
        bo, r = varint(v, 0, len(v))
        bs, r = varint(v, r, len(v))
        out.append((bo, bs))
        o = q + ns + vl
    return (ioff, isize), out


def reseal(t: bytearray, off: int, size: int):
    """Recompute the trailer checksum of the block at off after an edit."""
    crc = mask(crc32c_bitwise(bytes(t[off:off + size + 1])))
    t[off + size + 1:off + size + 5] = struct.pack("<I", crc)


def run(tables, job):
    return oracle.compact([bytes(t) for t in tables], job.options())


def test_clean_inputs_ok():
    job, ts = _tables()
    assert run(ts, job).status == 0


def test_checksum_error_location():
    job, ts = _tables()
    _, hs = handles(ts[1])
    k = len(hs) // 2
    bo, bs = hs[k]
    ts[1][bo + bs // 2] ^= 0x40
    r = run(ts, job)
    assert r.status == NAMES["CORRUPT_CHECKSUM"]
    assert (r.error.input, r.error.where, r.error.block, r.error.phase) == (1, 2, k, 0)


def test_first_error_wins_across_inputs_and_blocks():
    job, ts = _tables()
    _, h0 = handles(ts[0])
    _, h2 = handles(ts[2])
    # input 2 block 0 and input 0 last block: input 0 is reported
    ts[2][h2[0][0]] ^= 1
    bo, bs = h0[-1]
    ts[0][bo] ^= 1
    r = run(ts, job)
    assert (r.status, r.error.input, r.error.block) == (NAMES["CORRUPT_CHECKSUM"], 0, len(h0) - 1)
    # two blocks of one input: the earlier block is reported
    job, ts = _tables(seed=2)
    _, h1 = handles(ts[1])
    assert len(h1) >= 3
    ts[1][h1[2][0]] ^= 1
    ts[1][h1[1][0]] ^= 1
    r = run(ts, job)
    assert (r.error.input, r.error.block) == (1, 1)


def test_footer_errors():
    job, ts = _tables()
    t = bytes(ts[0])
    r = oracle.compact([t[:-1]] + [bytes(x) for x in ts[1:]], job.options())
    assert (r.status, r.error.input, r.error.where) == (NAMES["CORRUPT_FORMAT"], 0, 0)
    r = oracle.compact([bytes(x) for x in ts[:2]] + [b"\x00" * 20], job.options())
    assert (r.status, r.error.input, r.error.where, r.error.offset) == (NAMES["CORRUPT_FORMAT"], 2, 0, 0)
    bad = bytearray(t)
    bad[-1] ^= 0xFF
    r = oracle.compact([bytes(bad)], job.options())
    assert (r.status, r.error.where, r.error.offset) == (NAMES["CORRUPT_FORMAT"], 0, len(t) - 8)


def test_index_block_checksum_and_handle_range():
    job, ts = _tables()
    (io, isz), hs = handles(ts[1])
    t = bytearray(ts[1])
    t[io + 1] ^= 0x10
    r = oracle.compact([bytes(ts[0]), bytes(t)], job.options())
    assert (r.status, r.error.input, r.error.where) == (NAMES["CORRUPT_CHECKSUM"], 1, 1)


def test_unknown_block_type_unsupported():
    job, ts = _tables()
    _, hs = handles(ts[0])
    bo, bs = hs[0]
    ts[0][bo + bs] = 2  # block type 2: neither raw (0) nor Snappy (1)
    reseal(ts[0], bo, bs)
    r = run(ts, job)
    assert (r.status, r.error.input, r.error.where, r.error.block) == (NAMES["UNSUPPORTED"], 0, 2, 0)


def test_raw_contents_marked_snappy_are_a_bad_stream():
    # a raw block relabelled type 1: its first bytes (shared 0, non_shared,
    # value length varints) read as a Snappy preamble and elements, which
    # fail inside the block's stored bytes in the trailer phase
    job, ts = _tables()
    _, hs = handles(ts[0])
    bo, bs = hs[0]
    ts[0][bo + bs] = 1
    reseal(ts[0], bo, bs)
    r = run(ts, job)
    assert (r.status, r.error.input, r.error.where, r.error.block, r.error.phase) == \
        (NAMES["CORRUPT_FORMAT"], 0, 2, 0, 0)
    st, _, at = oracle.snappy_decompress(bytes(ts[0][bo:bo + bs]))
    assert st == NAMES["CORRUPT_FORMAT"] and r.error.offset == at


def test_restart_array_errors():
    job, ts = _tables()
    _, hs = handles(ts[0])
    bo, bs = hs[0]
    c = ts[0]
    nr = struct.unpack_from("<I", c, bo + bs - 4)[0]
    # num_restarts too large
    t = bytearray(c)
    t[bo + bs - 4:bo + bs] = struct.pack("<I", bs)
    reseal(t, bo, bs)
    r = oracle.compact([bytes(t)], job.options())
    assert (r.status, r.error.phase, r.error.offset) == (NAMES["CORRUPT_FORMAT"], 1, bs - 4)
    # first restart offset not zero
    t = bytearray(c)
    de = bs - 4 - 4 * nr
    t[bo + de:bo + de + 4] = struct.pack("<I", 1)
    reseal(t, bo, bs)
    r = oracle.compact([bytes(t)], job.options())
    assert (r.status, r.error.phase, r.error.offset) == (NAMES["CORRUPT_FORMAT"], 1, de)


def test_entry_errors_shared_at_restart_and_bad_type():
    job, ts = _tables()
    _, hs = handles(ts[0])
    bo, bs = hs[0]
    t = bytearray(ts[0])
    # first entry is a restart: make its shared count 1 (needs a one-byte varint)
    assert t[bo] == 0
    t[bo] = 1
    reseal(t, bo, bs)
    r = oracle.compact([bytes(t)], job.options())
    assert (r.status, r.error.phase, r.error.offset) == (NAMES["CORRUPT_FORMAT"], 2, 0)
    # type byte 7: the type sits 8 bytes from the end of the first internal key
    t = bytearray(ts[0])
    s, q = varint(t, bo, bo + bs, 5)
    ns, q = varint(t, q, bo + bs, 5)
    vl, q = varint(t, q, bo + bs, 5)
    t[q + ns - 8] = 7
    reseal(t, bo, bs)
    r = oracle.compact([bytes(t)], job.options())
    assert (r.status, r.error.phase, r.error.offset) == (NAMES["CORRUPT_FORMAT"], 2, 0)


def test_unsorted_input_reported_at_entry():
    # a table written from an out-of-order list decodes to UNSORTED_INPUT
    keys = [b"b", b"a", b"c"]
    tags = np.array([(5 << 8) | 1] * 3, np.uint64)
    koff = np.array([0, 1, 2, 3], np.uint64)
    voff = np.array([0, 0, 0, 0], np.uint64)
    opts = dict(block_size=4096, restart_interval=16, bloom_bits_per_key=10, bottommost=0,
                target_file_size=1 << 40)
    res = oracle.build_tables(np.frombuffer(b"bac", np.uint8), koff, tags, np.zeros(0, np.uint8),
                              voff, opts)
    t = res.files[0]
    r = oracle.compact([t], opts)
    assert (r.status, r.error.where, r.error.block, r.error.phase) == (NAMES["UNSORTED_INPUT"], 2, 0, 2)
    assert r.error.offset == 3 + 9  # second entry
    # equal internal keys inside one table are unsorted too
    res = oracle.build_tables(np.frombuffer(b"aa", np.uint8), np.array([0, 1, 2], np.uint64),
                              tags[:2], np.zeros(0, np.uint8), np.zeros(3, np.uint64), opts)
    r = oracle.compact([res.files[0]], opts)
    assert r.status == NAMES["UNSORTED_INPUT"]


def test_invalid_options():
    r = oracle.compact([], dict(block_size=0, restart_interval=16, bloom_bits_per_key=10,
                                bottommost=1, target_file_size=1))
    assert r.status == NAMES["INVALID_ARG"]
    r = oracle.compact([], dict(block_size=4096, restart_interval=0, bloom_bits_per_key=10,
                                bottommost=1, target_file_size=1))
    assert r.status == NAMES["INVALID_ARG"]
