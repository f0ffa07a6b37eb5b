"""An independent reader/validator of output tables (test helper).

Written separately from both the oracle and the GPU library: its own bitwise
CRC32C, its own varint and block parsing, and the `xxhash` package for Bloom
probes.  It checks every structural rule of the table layout:

* footer magic and handles; every block trailer (type 0, masked CRC32C of the
  contents and type byte);
* block entries: restart array, shared == 0 at restart points, shared prefix
  against the previous key, restart interval of the writer;
* index block: one entry per data block, key == the block's last internal key,
  value == the block's handle; blocks tile the data region;
* filter block: one filter per 2 KiB window up to the last block's window,
  each filter over exactly the user keys of the blocks starting in it, with no
  false negatives;
* block cut and file cut rules of the greedy writer.
"""
from __future__ import annotations

import struct
from dataclasses import dataclass
from typing import List, Optional, Tuple

import xxhash

MAGIC = 0xdb4775248b80fb57
FILTER_NAME = b"filter.luda.bloom.xxh64"


def crc32c_bitwise(data: bytes) -> int:
    crc = 0xFFFFFFFF
    for b in data:
        crc ^= b
        for _ in range(8):
            crc = (crc >> 1) ^ (0x82F63B78 if crc & 1 else 0)
    return crc ^ 0xFFFFFFFF


_T = []
for _b in range(256):
    _r = _b
    for _ in range(8):
        _r = (_r >> 1) ^ (0x82F63B78 if _r & 1 else 0)
    _T.append(_r)


def crc32c_fast(data: bytes) -> int:
    """Byte-table CRC32C (table derived above from the bitwise register update)."""
    r = 0xFFFFFFFF
    t = _T
    for b in data:
        r = t[(r ^ b) & 0xFF] ^ (r >> 8)
    return r ^ 0xFFFFFFFF


def mask(c: int) -> int:
    return (((c >> 15) | (c << 17)) + 0xa282ead8) & 0xFFFFFFFF


def varint(buf: bytes, pos: int, limit: int, maxlen: int = 10) -> Tuple[int, int]:
    v = 0
    for i in range(maxlen):
        if pos + i >= limit:
            raise ValueError("truncated varint")
        b = buf[pos + i]
        v |= (b & 0x7F) << (7 * i)
        if not b & 0x80:
            return v, pos + i + 1
    raise ValueError("varint too long")


def enc_varint(v: int) -> bytes:
    out = bytearray()
    while v >= 0x80:
        out.append((v & 0x7F) | 0x80)
        v >>= 7
    out.append(v)
    return bytes(out)


@dataclass
class Entry:
    ikey: bytes
    value: bytes
    shared: int
    size: int  # encoded bytes of the entry


@dataclass
class Block:
    offset: int
    size: int  # stored bytes (the handle's size)
    entries: List[Entry]
    restarts: List[int]
    raw_size: int = 0  # bytes of the raw contents


def snappy_decode(z: bytes) -> bytes:
    """A Snappy raw stream, decoded element by element (format description:
    varint32 length, then literals (tag & 3 == 0) and copies with 1-, 2- or
    4-byte offsets (tag & 3 == 1, 2, 3)); raises on any malformed element."""
    n, p = varint(z, 0, len(z), 5)
    out = bytearray()
    while p < len(z):
        tag = z[p]
        p += 1
        kind = tag & 3
        if kind == 0:
            ln = (tag >> 2) + 1
            if ln > 60:
                nb = ln - 60
                assert p + nb <= len(z), "literal length runs past the stream"
                ln = int.from_bytes(z[p:p + nb], "little") + 1
                p += nb
            assert p + ln <= len(z), "literal runs past the stream"
            out += z[p:p + ln]
            p += ln
            continue
        if kind == 1:
            assert p + 1 <= len(z)
            ln = 4 + ((tag >> 2) & 7)
            off = ((tag >> 5) << 8) | z[p]
            p += 1
        elif kind == 2:
            assert p + 2 <= len(z)
            ln = (tag >> 2) + 1
            off = int.from_bytes(z[p:p + 2], "little")
            p += 2
        else:
            assert p + 4 <= len(z)
            ln = (tag >> 2) + 1
            off = int.from_bytes(z[p:p + 4], "little")
            p += 4
        assert 0 < off <= len(out), "copy offset outside the bytes produced"
        for _ in range(ln):  # byte by byte: a copy may overlap what it writes
            out.append(out[-off])
    assert len(out) == n, "stream length differs from its preamble"
    return bytes(out)


def read_block(f: bytes, off: int, size: int, crc_fn=crc32c_fast, allow_snappy: bool = False) -> bytes:
    """A block's raw contents: type 0 stored as is; type 1 (data blocks of
    tables written with compression) a Snappy stream that saves at least an
    eighth of the raw bytes."""
    assert off + size + 5 <= len(f), "block beyond file"
    c = f[off:off + size]
    t = f[off + size]
    stored = struct.unpack_from("<I", f, off + size + 1)[0]
    assert t == 0 or (allow_snappy and t == 1), f"block type {t} not allowed here"
    assert stored == mask(crc_fn(f[off:off + size + 1])), "bad block checksum"
    if t == 1:
        raw = snappy_decode(c)
        assert len(c) < len(raw) - len(raw) // 8, "compressed form saves less than an eighth"
        return raw
    return c


def parse_entries(c: bytes) -> Tuple[List[Entry], List[int]]:
    assert len(c) >= 4
    nr = struct.unpack_from("<I", c, len(c) - 4)[0]
    assert 1 <= nr <= (len(c) - 4) // 4
    data_end = len(c) - 4 - 4 * nr
    restarts = list(struct.unpack_from(f"<{nr}I", c, data_end))
    ents = []
    o = 0
    prev = b""
    starts = []
    while o < data_end:
        starts.append(o)
        s, p = varint(c, o, data_end, 5)
        ns, p = varint(c, p, data_end, 5)
        vl, p = varint(c, p, data_end, 5)
        assert s <= len(prev)
        assert p + ns + vl <= data_end
        key = prev[:s] + c[p:p + ns]
        val = c[p + ns:p + ns + vl]
        ents.append(Entry(key, val, s, p + ns + vl - o))
        prev = key
        o = p + ns + vl
    assert o == data_end
    for r in restarts:
        assert r in starts, "restart offset not at an entry start"
        assert ents[starts.index(r)].shared == 0, "shared != 0 at a restart"
    return ents, restarts


def user_key(ikey: bytes) -> bytes:
    return ikey[:-8]


def tag_of(ikey: bytes) -> int:
    return struct.unpack("<Q", ikey[-8:])[0]


def ikey_lt(a: bytes, b: bytes) -> bool:
    ua, ub = user_key(a), user_key(b)
    if ua != ub:
        return ua < ub
    return tag_of(a) > tag_of(b)


def bloom_may_match(filt: bytes, key: bytes) -> bool:
    k = filt[-1]
    bits = (len(filt) - 1) * 8
    h = xxhash.xxh64_intdigest(key, 0)
    g, d = h & 0xFFFFFFFF, h >> 32
    for _ in range(k):
        pos = g % bits
        if not filt[pos >> 3] & (1 << (pos & 7)):
            return False
        g = (g + d) & 0xFFFFFFFF
    return True


@dataclass
class Table:
    blocks: List[Block]
    data_bytes: int
    filters: List[bytes]


def check_table(f: bytes, restart_interval: int, bits_per_key: int = 10,
                crc_fn=crc32c_fast, compression: int = 0) -> Table:
    """Validate one table; returns its parsed data blocks."""
    assert len(f) >= 48
    assert struct.unpack_from("<Q", f, len(f) - 8)[0] == MAGIC, "bad magic"
    ft = f[len(f) - 48:len(f) - 8]
    moff, p = varint(ft, 0, 40)
    msize, p = varint(ft, p, 40)
    ioff, p = varint(ft, p, 40)
    isize, p = varint(ft, p, 40)
    assert all(b == 0 for b in ft[p:]), "footer padding must be zero"
    # index
    ic = read_block(f, ioff, isize, crc_fn)
    ients, irest = parse_entries(ic)
    assert irest == [i for i in range(len(ic)) if i in irest]
    assert len(irest) == len(ients), "index restart interval must be 1"
    blocks: List[Block] = []
    pos = 0
    for ie in ients:
        boff, q = varint(ie.value, 0, len(ie.value))
        bsize, q = varint(ie.value, q, len(ie.value))
        assert q == len(ie.value)
        assert boff == pos, "data blocks must tile the data region"
        c = read_block(f, boff, bsize, crc_fn, allow_snappy=bool(compression))
        ents, rest = parse_entries(c)
        assert ents, "empty data block"
        # writer restart pattern: a restart every R entries, from entry 0
        starts = []
        o = 0
        for e in ents:
            starts.append(o)
            o += e.size
        exp = [starts[i] for i in range(0, len(ents), restart_interval)]
        assert rest == exp, "restart points must be every R entries"
        for i, e in enumerate(ents):
            if i % restart_interval:
                prev = ents[i - 1].ikey
                lcp = 0
                while lcp < min(len(prev), len(e.ikey)) and prev[lcp] == e.ikey[lcp]:
                    lcp += 1
                assert e.shared == lcp, "shared must be the full common prefix"
        assert ie.ikey == ents[-1].ikey, "index key must be the block's last key"
        blocks.append(Block(boff, bsize, ents, rest, len(c)))
        pos = boff + bsize + 5
    data_bytes = pos
    # metaindex -> filter
    mc = read_block(f, moff, msize, crc_fn)
    ments, _ = parse_entries(mc)
    assert len(ments) == 1 and ments[0].ikey == FILTER_NAME
    foff, q = varint(ments[0].value, 0, len(ments[0].value))
    fsize, q = varint(ments[0].value, q, len(ments[0].value))
    assert foff == data_bytes, "filter block follows the data blocks"
    assert moff == foff + fsize + 5 and ioff == moff + msize + 5 and ioff + isize + 5 == len(f) - 48
    fc = read_block(f, foff, fsize, crc_fn)
    assert fc[-1] == 11
    arr = struct.unpack_from("<I", fc, len(fc) - 5)[0]
    nf = (len(fc) - 5 - arr) // 4
    offs = list(struct.unpack_from(f"<{nf}I", fc, arr)) + [arr]
    assert nf == (blocks[-1].offset >> 11) + 1, "filters run to the last block's window"
    filters = [fc[offs[i]:offs[i + 1]] for i in range(nf)]
    for w in range(nf):
        keys = [user_key(e.ikey) for b in blocks if (b.offset >> 11) == w for e in b.entries]
        if not keys:
            assert filters[w] == b"", "empty window must have an empty filter"
            continue
        bits = max(64, len(keys) * bits_per_key)
        nbytes = (bits + 7) // 8
        assert len(filters[w]) == nbytes + 1
        k = min(30, max(1, bits_per_key * 69 // 100))
        assert filters[w][-1] == k
        for key in keys:
            assert bloom_may_match(filters[w], key), "Bloom false negative"
    return Table(blocks, data_bytes, filters)


def check_output(files: List[bytes], options: dict) -> List[Tuple[bytes, bytes]]:
    """Validate all output files and the cut rules; return (ikey, value) in order."""
    R = options["restart_interval"]
    bs = options["block_size"]
    target = options["target_file_size"]
    out = []
    tables = [check_table(f, R, options["bloom_bits_per_key"], compression=options.get("compression", 0))
              for f in files]
    nblocks_total = sum(len(t.blocks) for t in tables)
    bi = 0
    for ti, t in enumerate(tables):
        for b in t.blocks:
            bi += 1
            ents = b.entries
            sizes = [e.size for e in ents]
            c = len(ents)
            est_full = sum(sizes) + 4 * (-(-c // R)) + 4
            est_prev = sum(sizes[:-1]) + 4 * (-(-(c - 1) // R)) + 4 if c > 1 else None
            if est_prev is not None:
                assert est_prev < bs, "block should have been cut one entry earlier"
            if bi < nblocks_total:
                assert est_full >= bs, "block cut before reaching the block size"
            out.extend((e.ikey, e.value) for e in ents)
        last_block = t.blocks[-1].size + 5
        assert t.data_bytes - last_block < target, "file should have been cut one block earlier"
        if ti < len(tables) - 1:
            assert t.data_bytes >= target, "file cut before reaching the target size"
    for a, b in zip(out, out[1:]):
        assert ikey_lt(a[0], b[0]), "output internal keys must be strictly increasing"
        if not options.get("snapshots"):
            assert user_key(a[0]) < user_key(b[0]), "output user keys must be strictly increasing"
    return out
