"""Pins of the oracle's primitives against external definitions.

Each pin is something other than the oracle itself: published test vectors
(RFC 3720 for CRC32C), an independent library (python-xxhash for XXH64), a
bitwise definition, algebraic laws, or tables assembled byte by byte here.
"""
import os
import random
import struct

import numpy as np
import pytest
import xxhash

import oracle
from sstcheck import crc32c_bitwise, enc_varint, mask

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _inp(desc: str) -> bytes:
    if desc.startswith("ascii:"):
        return desc[6:].encode()
    if desc == "empty":
        return b""
    if desc == "00..1f":
        return bytes(range(32))
    if desc == "1f..00":
        return bytes(range(31, -1, -1))
    byte, n = desc.split("x")
    return bytes([int(byte, 16)]) * int(n)


def _vectors(name):
    for line in open(os.path.join(GOLD, name)):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        yield line.split()


def test_crc32c_rfc3720_vectors():
    n = 0
    for name, desc, exp in _vectors("crc32c_rfc3720.txt"):
        data = _inp(desc)
        assert oracle.crc32c(data) == int(exp, 16), name
        assert oracle.crc32c_bitwise(data) == int(exp, 16), name
        assert crc32c_bitwise(data) == int(exp, 16), name
        n += 1
    assert n == 5


def test_crc32c_table_equals_bitwise_random():
    rng = random.Random(7)
    for _ in range(200):
        b = bytes(rng.randrange(256) for _ in range(rng.randrange(0, 300)))
        assert oracle.crc32c(b) == oracle.crc32c_bitwise(b)


def test_crc32c_extend_law():
    rng = random.Random(8)
    for _ in range(100):
        a = bytes(rng.randrange(256) for _ in range(rng.randrange(0, 100)))
        b = bytes(rng.randrange(256) for _ in range(rng.randrange(0, 100)))
        assert oracle.crc32c_extend(oracle.crc32c(a), b) == oracle.crc32c(a + b)


def test_crc_mask():
    assert oracle.mask_crc(oracle.crc32c(b"123456789")) == 0xC78AB0E5
    rng = random.Random(9)
    for _ in range(1000):
        c = rng.randrange(1 << 32)
        assert oracle.unmask_crc(oracle.mask_crc(c)) == c
        assert oracle.mask_crc(c) == mask(c)


@pytest.mark.parametrize("v", [0, 1, 127, 128, (1 << 14) - 1, 1 << 14, (1 << 21) - 1, 1 << 21,
                               (1 << 28) - 1, 1 << 28, (1 << 32) - 1, 1 << 35, (1 << 63), (1 << 64) - 1])
def test_varint_roundtrip_and_boundaries(v):
    enc = oracle.put_varint64(v)
    assert enc == enc_varint(v)
    expected_len = max(1, -(-v.bit_length() // 7))
    assert len(enc) == expected_len
    assert oracle.get_varint64(enc) == (v, len(enc))
    if v < (1 << 32):
        assert oracle.get_varint32(enc) == (v, len(enc))
    else:
        assert oracle.get_varint32(enc) == (None, 0)


def test_varint_rejects():
    assert oracle.get_varint32(b"\x80\x80") == (None, 0)  # truncated
    assert oracle.get_varint32(b"\x80\x80\x80\x80\x80\x01") == (None, 0)  # 6 bytes
    assert oracle.get_varint32(b"\xff\xff\xff\xff\x10") == (None, 0)  # > 32 bits
    assert oracle.get_varint64(b"\xff" * 9 + b"\x02") == (None, 0)  # > 64 bits
    assert oracle.get_varint64(b"") == (None, 0)


def test_xxh64_golden_vectors():
    n = 0
    for desc, exp in _vectors("xxh64_vectors.txt"):
        data = _inp(desc)
        assert oracle.xxh64(data) == int(exp, 16), desc
        assert xxhash.xxh64_intdigest(data) == int(exp, 16), desc
        n += 1
    assert n == 4


def test_xxh64_vs_library_random():
    rng = np.random.default_rng(10)
    for n in list(range(0, 70)) + [100, 127, 128, 129, 255, 1000]:
        for _ in range(3):
            b = rng.bytes(n)
            for seed in (0, 1, 0xDEADBEEFCAFEBABE):
                assert oracle.xxh64(b, seed) == xxhash.xxh64_intdigest(b, seed)


def test_bloom_size_rule():
    # bits = max(64, n * b) rounded up to bytes, plus one byte holding k
    assert oracle.bloom_size(0) == 9
    assert oracle.bloom_size(1) == 9
    assert oracle.bloom_size(6) == 9
    assert oracle.bloom_size(7) == 10   # 70 bits -> 9 bytes
    assert oracle.bloom_size(33) == 43  # 330 bits -> 42 bytes
    assert oracle.bloom_size(1000) == 1251
    f = oracle.bloom_build([b"x"])
    assert f[-1] == 6  # k = 10 * 69 // 100


def test_bloom_bits_with_library_hash():
    # the probe sequence recomputed with the independent xxhash library
    keys = [bytes([i]) * (i % 7 + 1) for i in range(40)]
    f = oracle.bloom_build(keys)
    bits = (len(f) - 1) * 8
    exp = bytearray(len(f) - 1)
    for k in keys:
        h = xxhash.xxh64_intdigest(k, 0)
        g, d = h & 0xFFFFFFFF, h >> 32
        for _ in range(6):
            p = g % bits
            exp[p >> 3] |= 1 << (p & 7)
            g = (g + d) & 0xFFFFFFFF
    assert f[:-1] == bytes(exp)


def test_bloom_no_false_negatives_and_fpr():
    rng = np.random.default_rng(11)
    n = 2000
    keys = [rng.bytes(16) for _ in range(n)]
    f = oracle.bloom_build(keys)
    for k in keys:
        assert oracle.bloom_may_match(f, k)
    absent = [rng.bytes(17) for _ in range(100_000)]
    fp = sum(oracle.bloom_may_match(f, k) for k in absent)
    k = 6
    theory = (1 - np.exp(-k / 10.0)) ** k  # asymptotic FPR at 10 bits/key, k = 6
    rate = fp / len(absent)
    assert 0.5 * theory <= rate <= 2.0 * theory, (rate, theory)


# --------------------------------------------------------------------------
# hand-assembled tables, written byte by byte from the layout rules


def _trailer(contents: bytes, btype: int = 0) -> bytes:
    return contents + bytes([btype]) + struct.pack("<I", mask(crc32c_bitwise(contents + bytes([btype]))))


def _block(entries, restarts):
    body = b""
    for shared, delta, val in entries:
        body += enc_varint(shared) + enc_varint(len(delta)) + enc_varint(len(val)) + delta + val
    return body + b"".join(struct.pack("<I", r) for r in restarts) + struct.pack("<I", len(restarts))


def _ikey(uk: bytes, seq: int, typ: int) -> bytes:
    return uk + struct.pack("<Q", (seq << 8) | typ)


def _table(data_blocks_entries, restarts_list):
    """Assemble a table from data-block entry lists; empty filter/metaindex."""
    out = b""
    handles = []
    last_keys = []
    for ents, rs in zip(data_blocks_entries, restarts_list):
        c = _block(ents, rs)
        handles.append((len(out), len(c)))
        key = b""
        for s, d, _ in ents:
            key = key[:s] + d
        last_keys.append(key)
        out += _trailer(c)
    # the metaindex of an input is never read by a compaction: a bare
    # restart array stands in for it
    meta = struct.pack("<II", 0, 1)
    moff = len(out)
    out += _trailer(meta)
    iblk_entries = []
    for (o, s), k in zip(handles, last_keys):
        iblk_entries.append((0, k, enc_varint(o) + enc_varint(s)))
    ioff = len(out)
    ic = _block(iblk_entries, list(_offsets(iblk_entries)))
    out += _trailer(ic)
    footer = enc_varint(moff) + enc_varint(len(meta)) + enc_varint(ioff) + enc_varint(len(ic))
    footer += bytes(40 - len(footer)) + struct.pack("<Q", 0xdb4775248b80fb57)
    return out + footer


def _offsets(entries):
    o = 0
    for s, d, v in entries:
        yield o
        o += len(enc_varint(s)) + len(enc_varint(len(d))) + len(enc_varint(len(v))) + len(d) + len(v)


def test_decode_hand_built_table():
    k1, k2, k3, k4 = _ikey(b"apple", 9, 1), _ikey(b"apply", 7, 1), _ikey(b"banana", 5, 0), _ikey(b"band", 4, 1)
    # restart interval 2: entries 0 and 2 are restarts
    e = [(0, k1, b"v1"), (4, k2[4:], b"vv2"), (0, k3, b""), (3, k4[3:], b"v4")]
    offs = list(_offsets(e))
    t = _table([e], [[offs[0], offs[2]]])
    st, err, dec = oracle.decode_table(t)
    assert st == 0, err
    keys, tags, vals = dec
    assert keys == [b"apple", b"apply", b"banana", b"band"]
    assert [int(x) for x in tags] == [(9 << 8) | 1, (7 << 8) | 1, (5 << 8) | 0, (4 << 8) | 1]
    assert vals == [b"v1", b"vv2", b"", b"v4"]


def test_decode_two_blocks_and_cross_block_order():
    a = [(0, _ikey(b"a", 3, 1), b"x")]
    b = [(0, _ikey(b"b", 2, 1), b"y"), (1, _ikey(b"b", 1, 0)[1:], b"")]
    t = _table([a, b], [[0], [0]])
    st, err, dec = oracle.decode_table(t)
    assert st == 0, err
    assert dec[0] == [b"a", b"b", b"b"]
    # same user key, tags must descend: swapping the versions is unsorted
    b_bad = [(0, _ikey(b"b", 1, 1), b"y"), (1, _ikey(b"b", 2, 0)[1:], b"")]
    st, err, _ = oracle.decode_table(_table([a, b_bad], [[0], [0]]))
    assert oracle.STATUS_NAMES[st] == "UNSORTED_INPUT"
    assert (err.where, err.block, err.phase) == (2, 1, 2)
    assert err.offset == len(enc_varint(0)) * 2 + 1 + 9 + 1  # second entry of block 1


def test_encode_decode_roundtrip_against_hand_layout():
    # a table written by the oracle must decode, through the independent
    # checker, to exactly the entries given
    from sstcheck import check_table
    keys = [b"k%03d" % i for i in range(50)]
    tags = np.array([((100 - i) << 8) | (i % 2) for i in range(50)], np.uint64)
    vals = [bytes([i]) * (i % 13) for i in range(50)]
    koff = np.cumsum([0] + [len(k) for k in keys]).astype(np.uint64)
    voff = np.cumsum([0] + [len(v) for v in vals]).astype(np.uint64)
    opts = dict(block_size=64, restart_interval=3, bloom_bits_per_key=10, bottommost=0,
                target_file_size=1 << 40)
    res = oracle.build_tables(np.frombuffer(b"".join(keys), np.uint8), koff, tags,
                              np.frombuffer(b"".join(vals), np.uint8), voff, opts)
    assert res.status == 0 and len(res.files) == 1
    tb = check_table(res.files[0], 3)
    got = [(e.ikey, e.value) for b in tb.blocks for e in b.entries]
    assert got == [(keys[i] + struct.pack("<Q", int(tags[i])), vals[i]) for i in range(50)]
    st, err, dec = oracle.decode_table(res.files[0])
    assert st == 0 and dec[0] == keys and dec[2] == vals
