"""Pins of the oracle's block compression (block type 1, Snappy raw streams).

* Decoding: streams assembled byte by byte here from the public format
  description (literals with inline and 1-4 extra length bytes; copies in the
  1-, 2- and 4-byte offset forms; overlapping copies), and malformed streams
  with the error offset each must report.
* Encoding: every stream decodes back (by the oracle and by the independent
  decoder in sstcheck) to its input; closed forms of the writer's rules on
  inputs whose streams can be worked out by hand (incompressible bytes, a
  zero run, a periodic run; the copy-splitting rule).
* Tables: with compression on, a table's blocks are type 1 exactly when the
  stream saves an eighth, and a compaction's outputs read back (sstcheck) to
  the same entries as without compression.
"""
import numpy as np
import pytest

import oracle
import sstcheck
from workload import compressible, plain_small, tiny_job


def varint(v: int) -> bytes:
    out = bytearray()
    while v >= 0x80:
        out.append((v & 0x7F) | 0x80)
        v >>= 7
    out.append(v)
    return bytes(out)


def lit(b: bytes) -> bytes:
    """A literal element, assembled from the format description."""
    m = len(b) - 1
    if m < 60:
        return bytes([m << 2]) + b
    nb = (m.bit_length() + 7) // 8
    return bytes([(59 + nb) << 2]) + m.to_bytes(nb, "little") + b


def copy1(off: int, n: int) -> bytes:
    assert 4 <= n <= 11 and off < 2048
    return bytes([1 | ((n - 4) << 2) | ((off >> 8) << 5), off & 0xFF])


def copy2(off: int, n: int) -> bytes:
    assert 1 <= n <= 64 and off < 65536
    return bytes([2 | ((n - 1) << 2)]) + off.to_bytes(2, "little")


def copy4(off: int, n: int) -> bytes:
    assert 1 <= n <= 64
    return bytes([3 | ((n - 1) << 2)]) + off.to_bytes(4, "little")


HAND = [
    (varint(5) + lit(b"hello"), b"hello"),
    (varint(0), b""),
    (varint(100) + lit(bytes(range(100))), bytes(range(100))),                       # 1 extra length byte
    (varint(300) + lit(bytes(300)), bytes(300)),                                      # 2 extra length bytes
    (varint(12) + lit(b"abcd") + copy1(4, 8), b"abcdabcdabcd"),                       # overlapping 1-byte form
    (varint(11) + lit(b"a") + copy1(1, 10), b"a" * 11),                               # offset 1: a run
    (varint(70) + lit(b"xyz") + copy2(3, 64) + copy2(2, 3), None),                  # 2-byte form, period 3
    (varint(9) + lit(b"12345") + copy4(5, 4), b"123451234"),                          # 4-byte offset form
    (varint(2058) + lit(bytes([7]) * 2048 + b"QRST") + copy1(2047, 4) + lit(b"zz"),
     bytes([7]) * 2048 + b"QRST" + bytes([7]) * 4 + b"zz"),                           # largest 11-bit offset
]


def _period_case():
    # "xyz", then 64 bytes copied from 3 back, then 3 bytes copied from 2 back,
    # produced one byte at a time as the format defines an overlapping copy
    s = bytearray(b"xyz")
    for _ in range(64):
        s.append(s[-3])
    for _ in range(3):
        s.append(s[-2])
    return bytes(s)


HAND[6] = (HAND[6][0], _period_case())


@pytest.mark.parametrize("k", range(len(HAND)))
def test_hand_streams_decode(k):
    stream, want = HAND[k]
    assert len(want) == sstcheck.varint(stream, 0, len(stream))[0]
    st, got, _ = oracle.snappy_decompress(stream)
    assert st == 0 and got == want
    assert sstcheck.snappy_decode(stream) == want


BAD = [
    (b"", 0),                                            # no preamble
    (b"\x80\x80\x80\x80\x80\x01", 0),                    # preamble longer than 5 bytes
    (b"\xff\xff\xff\xff\x1f", 0),                        # preamble above 32 bits
    (varint(4) + bytes([3 << 2]) + b"abc", 1),           # literal runs past the stream
    (varint(8) + bytes([60 << 2]), 1),                   # literal's length byte missing
    (varint(3) + lit(b"abcd"), 1),                       # literal longer than the declared length
    (varint(6) + lit(b"ab") + copy1(0, 4), 4),           # offset 0
    (varint(7) + lit(b"ab") + copy2(3, 4), 4),           # offset beyond the bytes produced
    (varint(7) + lit(b"ab") + copy2(2, 6), 4),           # copy past the declared length
    (varint(6) + lit(b"ab") + bytes([2 | (3 << 2), 2]), 4),  # 2-byte offset cut short
    (varint(6) + lit(b"ab") + bytes([3 | (3 << 2), 2, 0, 0]), 4),  # 4-byte offset cut short
    (varint(6) + lit(b"ab") + bytes([1 | (0 << 2)]), 4),  # 1-byte offset missing
    (varint(9) + lit(b"abc") + copy1(3, 4), 7),          # stream ends short of the declared length
]


@pytest.mark.parametrize("k", range(len(BAD)))
def test_malformed_streams(k):
    stream, at = BAD[k]
    st, got, off = oracle.snappy_decompress(stream)
    assert st == oracle.STATUS_CODES["CORRUPT_FORMAT"] and got is None
    assert off == at
    with pytest.raises((AssertionError, ValueError)):
        sstcheck.snappy_decode(stream)


def test_incompressible_bytes_are_one_literal():
    # no 4-byte string repeats, so the stream is the preamble and one literal
    rng = np.random.default_rng(1)
    for n in (1, 3, 4, 59, 60, 61, 256, 257, 4096, 65536):
        while True:
            b = rng.bytes(n)
            if len({b[i:i + 4] for i in range(max(0, n - 3))}) == max(0, n - 3):
                break
        assert oracle.snappy_compress(b) == varint(n) + lit(b), n


def test_zero_run_closed_form():
    # the first group of 64 positions finds an empty table: 64 literal bytes;
    # position 64 finds position 63 (the last of group 0 under the same hash):
    # one copy at offset 1 to the end, split 64, 64, ..., then the rest
    for n in (65, 67):  # position 64 has fewer than 4 bytes left: no lookup
        assert oracle.snappy_compress(bytes(n)) == varint(n) + lit(bytes(n)), n
    for n in (68, 75, 128, 131, 132, 4096, 65536):
        L = n - 64
        pieces = b""
        while L >= 68:
            pieces += copy2(1, 64)
            L -= 64
        if L > 64:
            pieces += copy2(1, 60)
            L -= 60
        pieces += copy1(1, L) if L <= 11 else copy2(1, L)
        assert oracle.snappy_compress(bytes(n)) == varint(n) + lit(bytes(64)) + pieces, n


def test_periodic_run_uses_the_last_earlier_position():
    # period 8: position 64 looks up the last of 0, 8, ..., 56 (56): offset 8
    pat = b"ABCDEFGH"
    b = pat * 40  # 320 bytes: 64 literal, then 256 copied from 8 back
    want = varint(len(b)) + lit(b[:64]) + copy2(8, 64) * 4
    assert oracle.snappy_compress(b) == want
    b = pat * 9  # 72 bytes: 64 literal, then 8 copied in the 2-byte form
    assert oracle.snappy_compress(b) == varint(72) + lit(b[:64]) + copy1(8, 8)


def test_fragments_of_64_kib_are_compressed_separately():
    # two identical 64 KiB fragments of random bytes: no copy may reach back
    # into the first one, so both are single literals
    frag = np.random.default_rng(2).bytes(65536)
    z = oracle.snappy_compress(frag + frag)
    assert z == varint(131072) + lit(frag) + lit(frag)


@pytest.mark.parametrize("seed", range(6))
def test_round_trip(seed):
    rng = np.random.default_rng(seed)
    for n in (0, 1, 17, 1000, 4096, 20000, 70000, 140000):
        kind = rng.integers(0, 3)
        if kind == 0:
            b = rng.bytes(n)
        elif kind == 1:
            b = bytes(rng.integers(0, 4, n, dtype=np.uint8))
        else:
            words = [rng.bytes(int(rng.integers(1, 9))) for _ in range(20)]
            b = b"".join(words[int(i)] for i in rng.integers(0, 20, n))[:n]
        z = oracle.snappy_compress(b)
        assert len(z) <= oracle.lib().ref_snappy_max(len(b))
        st, back, _ = oracle.snappy_decompress(z)
        assert st == 0 and back == b
        assert sstcheck.snappy_decode(z) == b


def _blocks(table: bytes):
    t = sstcheck.check_table(table, 16, compression=1)
    return [(b.offset, b.size, b.raw_size, table[b.offset + b.size]) for b in t.blocks]


def test_compressed_tables_store_a_block_compressed_iff_it_saves_an_eighth():
    job = compressible(plain_small())
    ins = oracle.build_input_tables(job)
    types = [x[3] for t in ins for x in _blocks(t)]
    assert 0 < types.count(1) < len(types), "the variant should mix compressed and raw blocks"
    for t in ins:
        for off, size, raw, typ in _blocks(t):
            raw_block = sstcheck.read_block(t, off, size, allow_snappy=True)
            z = oracle.snappy_compress(raw_block)
            assert (typ == 1) == (len(z) < raw - raw // 8)
            if typ == 1:
                assert t[off:off + size] == z


@pytest.mark.parametrize("make", [lambda: compressible(plain_small()),
                                  lambda: compressible(tiny_job(3, entries=400, val_len=(0, 300),
                                                                block_size=512, target_file_size=4096), 3)])
def test_compaction_with_compression_reads_back_the_same(make):
    job = make()
    ins = oracle.build_input_tables(job)
    res = oracle.compact(ins, job.options())
    assert res.status == 0
    plain = dict(job.options())
    plain.pop("compression")
    ref = oracle.compact(ins, plain)  # compressed inputs, raw outputs
    assert ref.status == 0
    assert sstcheck.check_output(res.files, job.options()) == sstcheck.check_output(ref.files, plain)
    assert (res.entries_in, res.entries_out) == (ref.entries_in, ref.entries_out)
    assert sum(map(len, res.files)) < sum(map(len, ref.files))


def test_index_blocks_must_be_stored_raw():
    # a type-1 trailer on the index block is refused (only data blocks may be
    # compressed); the checksum is made valid so the type is what fails
    job = tiny_job(1, entries=60)
    t = bytearray(oracle.build_input_tables(job)[0])
    ft = t[-48:-8]
    _m, p = sstcheck.varint(ft, 0, 40)
    _m, p = sstcheck.varint(ft, p, 40)
    ioff, p = sstcheck.varint(ft, p, 40)
    isize, p = sstcheck.varint(ft, p, 40)
    t[ioff + isize] = 1
    crc = oracle.crc32c(bytes(t[ioff:ioff + isize + 1]))
    t[ioff + isize + 1:ioff + isize + 5] = oracle.mask_crc(crc).to_bytes(4, "little")
    st, err, _ = oracle.decode_table(bytes(t))
    assert st == oracle.STATUS_CODES["UNSUPPORTED"] and (err.where, err.phase) == (1, 0)


def _first_copy(z: bytes) -> int:
    """Offset of the first copy element of a stream (walked from the format)."""
    _n, p = sstcheck.varint(z, 0, len(z), 5)
    while p < len(z):
        tag = z[p]
        if tag & 3:
            return p
        ln = (tag >> 2) + 1
        extra = 0
        if ln > 60:
            extra = ln - 60
            ln = int.from_bytes(z[p + 1:p + 1 + extra], "little") + 1
        p += 1 + extra + ln
    raise AssertionError("no copy element")


def test_a_bad_copy_in_a_data_block_is_reported_at_its_element():
    job = compressible(plain_small())
    t = bytearray(oracle.build_input_tables(job)[1])
    blocks = sstcheck.check_table(bytes(t), 16, compression=1).blocks
    k = next(i for i, b in enumerate(blocks) if t[b.offset + b.size] == 1 and i > 2)
    b = blocks[k]
    z = bytes(t[b.offset:b.offset + b.size])
    at = _first_copy(z)
    kind = z[at] & 3
    if kind == 1:  # offset 0 in the 1-byte form: clear the tag's high bits and the byte
        t[b.offset + at] &= 0x1F
        t[b.offset + at + 1] = 0
    else:
        t[b.offset + at + 1:b.offset + at + 1 + (2 if kind == 2 else 4)] = bytes(2 if kind == 2 else 4)
    crc = oracle.crc32c(bytes(t[b.offset:b.offset + b.size + 1]))
    t[b.offset + b.size + 1:b.offset + b.size + 5] = oracle.mask_crc(crc).to_bytes(4, "little")
    st, err, _ = oracle.decode_table(bytes(t), 1)
    assert st == oracle.STATUS_CODES["CORRUPT_FORMAT"]
    assert (err.input, err.where, err.phase, err.block, err.offset) == (1, 2, 0, k, at)


def test_worst_case_expansion_stays_within_the_bound():
    # 61 random bytes, then 4 bytes repeated from 2080 back (a 3-byte copy
    # when it is found): such a pair costs 2 + 61 + 3 bytes for 65 raw bytes
    rng = np.random.default_rng(5)
    b = bytearray(rng.bytes(200000))
    for i in range(2080 // 65 + 1, len(b) // 65):
        p = 65 * i + 61
        b[p:p + 4] = b[p - 2080:p - 2076]
    b = bytes(b)
    z = oracle.snappy_compress(b)
    assert len(z) > len(b)  # it does expand
    assert len(z) <= oracle.lib().ref_snappy_max(len(b))
    st, back, _ = oracle.snappy_decompress(z)
    assert st == 0 and back == b
