"""Seeded generators for the logical content of compaction inputs.

A compaction job merges one upper-level table with the lower-level tables whose
key ranges overlap it (paper, Sec. II-A: level i tables are merged into level
i+1).  The paper evaluates with 16-byte keys, 128 B - 1 KiB values, 4 KiB data
blocks, 4 MiB tables and 10-bit/key Bloom filters (Sec. IV-A).  These
generators stand in for the YCSB-loaded LevelDB tables of that evaluation: no
YCSB data or trace is reproduced, only synthetic keys and values of the stated
shapes.

Everything here is the input side only.  A :class:`Run` holds one input
table's entries as sorted, typed key/value records; turning it into table bytes
is the job of whichever side consumes it (the oracle's table writer, or the GPU
library's own writer).

Conventions shared by every workload:

* internal key order inside a run: user key ascending (bytewise, shorter key
  first on a common prefix), then tag descending, where
  ``tag = (sequence << 8) | type`` and type 1 = value, 0 = deletion;
* sequence numbers are < 2**56 and increase with level recency: lower-level
  entries get ``2**52 + pi(r)`` and upper-level entries ``2**54 + pi(r)``, with
  ``pi`` a seeded permutation of entry ranks (uncorrelated with key order);
* deletions (tombstones) carry an empty value;
* 16-byte keys are ``BE64(fmix64(id ^ salt)) || BE64(id)`` where fmix64 is the
  SplitMix64 finaliser (Steele, Lea & Flood, OOPSLA 2014), a bijection, so
  distinct ids give distinct keys spread uniformly in byte order.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

TYPE_DELETION = 0
TYPE_VALUE = 1

SEED_BASE = 0x4C554441  # "LUDA"
MiB = 1 << 20
_U64 = np.uint64


def workload_seed(workload: int, job: int = 0) -> int:
    """Default seed of a workload (0 plain small, 1 plain large, 2 plain
    variable, 3 batch) and of one job of it."""
    return SEED_BASE ^ (workload << 32) ^ job


@dataclass
class Run:
    """One input table's logical content, sorted in internal key order."""

    keys: np.ndarray  # uint8, concatenated user keys
    koff: np.ndarray  # int64, n+1 offsets into keys
    tags: np.ndarray  # uint64, n tags (seq << 8 | type)
    vals: np.ndarray  # uint8, concatenated values
    voff: np.ndarray  # int64, n+1 offsets into vals

    @property
    def n(self) -> int:
        return int(self.tags.shape[0])

    def key(self, i: int) -> bytes:
        return self.keys[self.koff[i]:self.koff[i + 1]].tobytes()

    def value(self, i: int) -> bytes:
        return self.vals[self.voff[i]:self.voff[i + 1]].tobytes()

    def entries(self):
        """Yield (user_key, tag, value) tuples (slow; small runs only)."""
        for i in range(self.n):
            yield self.key(i), int(self.tags[i]), self.value(i)

    def approx_bytes(self) -> int:
        """Logical payload size: key + 8-byte tag + value + 4 per entry."""
        return int(self.keys.size + self.vals.size + 12 * self.n)


@dataclass
class Job:
    """One compaction: runs[0] is the upper (newest) table, then the lower ones."""

    runs: List[Run]
    block_size: int = 4096
    restart_interval: int = 16
    bloom_bits_per_key: int = 10
    bottommost: int = 1
    target_file_size: int = 2 * MiB
    name: str = ""
    meta: dict = field(default_factory=dict)
    compression: int = 0  # 1: data blocks stored as Snappy streams when that saves >= 1/8

    def options(self) -> dict:
        o = dict(block_size=self.block_size, restart_interval=self.restart_interval,
                 bloom_bits_per_key=self.bloom_bits_per_key, bottommost=self.bottommost,
                 target_file_size=self.target_file_size)
        if self.compression:
            o["compression"] = self.compression
        return o

    def table_options(self) -> dict:
        """Options for writing this job's *input* tables (one file per run)."""
        o = self.options()
        o["target_file_size"] = 1 << 62
        o["bottommost"] = 0
        return o


# ----------------------------------------------------------------------------
# small helpers


def fmix64(x: np.ndarray) -> np.ndarray:
    """SplitMix64 finaliser (a bijection on 64-bit words)."""
    x = x.astype(_U64, copy=True)
    with np.errstate(over="ignore"):
        x ^= x >> _U64(30)
        x *= _U64(0xBF58476D1CE4E5B9)
        x ^= x >> _U64(27)
        x *= _U64(0x94D049BB133111EB)
        x ^= x >> _U64(31)
    return x


def mix32(x: np.ndarray, salt: int) -> np.ndarray:
    """A seeded bijection on 32-bit words (xor-shift / odd-multiply rounds)."""
    x = (x.astype(np.uint64) ^ np.uint64(salt & 0xFFFFFFFF)) & np.uint64(0xFFFFFFFF)
    m = np.uint64(0xFFFFFFFF)
    with np.errstate(over="ignore"):
        x ^= x >> np.uint64(16)
        x = (x * np.uint64(0x7FEB352D)) & m
        x ^= x >> np.uint64(15)
        x = (x * np.uint64(0x846CA68B)) & m
        x ^= x >> np.uint64(16)
    return x


def key16(ids: np.ndarray, salt: int) -> np.ndarray:
    """(n, 16) uint8 keys: BE64(fmix64(id ^ salt)) || BE64(id)."""
    ids = ids.astype(_U64)
    hi = fmix64(ids ^ _U64(salt & 0xFFFFFFFFFFFFFFFF))
    out = np.empty((ids.shape[0], 2), dtype=">u8")
    out[:, 0] = hi
    out[:, 1] = ids
    return out.view(np.uint8).reshape(ids.shape[0], 16)


def zipf_rejection_inversion(rng: np.random.Generator, n: int, N: float, s: float) -> np.ndarray:
    """Draw Zipf(s) ranks in [1, N] by rejection-inversion.

    Method of Hoermann & Derflinger, "Rejection-inversion to generate variates
    from monotone discrete distributions", ACM TOMACS 6(3), 1996.  Returns the
    accepted draws (a little fewer than n).
    """
    one_s = 1.0 - s

    def H(x):
        return np.expm1(one_s * np.log(x)) / one_s

    def Hinv(y):
        return np.exp(np.log1p(y * one_s) / one_s)

    def h(x):
        return np.exp(-s * np.log(x))

    H_x1 = H(1.5) - 1.0
    H_n = H(N + 0.5)
    thr = 2.0 - Hinv(H(2.5) - h(2.0))
    u = H_n + rng.random(n) * (H_x1 - H_n)
    x = Hinv(u)
    k = np.clip(np.floor(x + 0.5), 1.0, N)
    acc = (k - x <= thr) | (u >= H(k + 0.5) - h(k))
    return k[acc].astype(np.uint64)


def _values(rng: np.random.Generator, vlens: np.ndarray):
    voff = np.zeros(vlens.shape[0] + 1, dtype=np.int64)
    np.cumsum(vlens, out=voff[1:])
    total = int(voff[-1])
    vals = np.frombuffer(rng.bytes(total), dtype=np.uint8) if total else np.zeros(0, np.uint8)
    return vals, voff


def _run_from_fixed(keys2d: np.ndarray, tags: np.ndarray, vlens: np.ndarray,
                    rng: np.random.Generator) -> Run:
    n, w = keys2d.shape
    koff = np.arange(n + 1, dtype=np.int64) * w
    vals, voff = _values(rng, vlens)
    return Run(np.ascontiguousarray(keys2d).reshape(-1), koff, tags.astype(_U64), vals, voff)


def _seqs(rng: np.random.Generator, n: int, base: int) -> np.ndarray:
    return _U64(base) + rng.permutation(n).astype(_U64)


def _tags(seqs: np.ndarray, types: np.ndarray) -> np.ndarray:
    return (seqs.astype(_U64) << _U64(8)) | types.astype(_U64)


def _split_counts(total: int, parts: int) -> List[int]:
    base = total // parts
    rem = total - base * parts
    return [base + (1 if i < rem else 0) for i in range(parts)]


def _fixed_level(rng, ids_sorted_keys, n_files_sizes, seq_base, vlen_fn, p_tomb):
    """Split one sorted distinct key set into consecutive files."""
    n = ids_sorted_keys.shape[0]
    seqs = _seqs(rng, n, seq_base)
    types = (rng.random(n) >= p_tomb).astype(np.uint8)
    vlens = np.where(types == TYPE_VALUE, vlen_fn(n), 0).astype(np.int64)
    runs = []
    start = 0
    for cnt in n_files_sizes:
        sl = slice(start, start + cnt)
        runs.append(_run_from_fixed(ids_sorted_keys[sl], _tags(seqs[sl], types[sl]), vlens[sl], rng))
        start += cnt
    return runs


def _sorted_key16(ids: np.ndarray, salt: int) -> np.ndarray:
    k = key16(ids, salt)
    w = k.view(">u8").reshape(-1, 2)
    order = np.lexsort((w[:, 1], w[:, 0]))
    return k[order]


# ----------------------------------------------------------------------------
# plain small: one compaction of three small tables


def plain_small(seed: Optional[int] = None) -> Job:
    """1 upper table (10,000 entries) + 2 disjoint lower tables (10,000 each).

    Ids uniform over [0, 2**20) so upper/lower duplicates occur; 100-byte
    values; 5% tombstones; 4 KiB blocks, restart interval 16, 10 bits/key;
    output split at 2 MiB; bottom level (tombstones dropped).
    """
    seed = workload_seed(0) if seed is None else seed
    rng = np.random.default_rng(seed)
    salt = int(rng.integers(0, 2**63))
    lower_ids = rng.choice(1 << 20, 20000, replace=False)
    upper_ids = rng.choice(1 << 20, 10000, replace=False)
    fixed = lambda n: np.full(n, 100, np.int64)  # noqa: E731
    upper = _fixed_level(rng, _sorted_key16(upper_ids, salt), [10000], 1 << 54, fixed, 0.05)
    lower = _fixed_level(rng, _sorted_key16(lower_ids, salt), [10000, 10000], 1 << 52, fixed, 0.05)
    return Job(upper + lower, block_size=4096, restart_interval=16, bloom_bits_per_key=10,
               bottommost=1, target_file_size=2 * MiB, name="plain-small-3x10k-v100")


# ----------------------------------------------------------------------------
# plain large: Zipf 0.99 over 2**32, 1 KiB values


def _draw_distinct_zipf(rng, count: int, salt32: int, exclude=None) -> np.ndarray:
    got = np.zeros(0, dtype=np.uint64)
    while got.shape[0] < count:
        need = count - got.shape[0]
        ranks = zipf_rejection_inversion(rng, max(4 * need, 1024), float(2**32), 0.99)
        ids = mix32(ranks - np.uint64(1), salt32)
        got = np.unique(np.concatenate([got, ids]))
    # keep a seeded subset of exactly `count` distinct ids
    return rng.choice(got, count, replace=False)


def plain_large(seed: Optional[int] = None, scale: float = 1.0) -> Job:
    """1 upper + 10 lower tables of ~64 MiB each (~700 MiB input).

    16-byte keys whose ids are Zipf(0.99)-distributed ranks over [1, 2**32]
    mapped through a seeded 32-bit bijection; 1 KiB values; 2% tombstones;
    not the bottom level (tombstones kept); 4 KiB blocks; 64 MiB output files.
    ``scale`` shrinks the table sizes for quick runs.
    """
    seed = workload_seed(1) if seed is None else seed
    rng = np.random.default_rng(seed)
    salt = int(rng.integers(0, 2**63))
    salt32 = int(rng.integers(0, 2**32))
    per_file = max(16, int(round((64 * MiB * scale) / (16 + 8 + 1024 + 4))))
    upper_ids = _draw_distinct_zipf(rng, per_file, salt32)
    lower_ids = _draw_distinct_zipf(rng, 10 * per_file, salt32)
    v1k = lambda n: np.full(n, 1024, np.int64)  # noqa: E731
    upper = _fixed_level(rng, _sorted_key16(upper_ids, salt), [per_file], 1 << 54, v1k, 0.02)
    lower = _fixed_level(rng, _sorted_key16(lower_ids, salt), _split_counts(10 * per_file, 10),
                         1 << 52, v1k, 0.02)
    return Job(upper + lower, block_size=4096, restart_interval=16, bloom_bits_per_key=10,
               bottommost=0, target_file_size=max(1, int(64 * MiB * scale)),
               name=f"plain-large-11x{64 * scale:g}MiB-zipf0.99-v1024")


# ----------------------------------------------------------------------------
# plain variable: variable-size keys and values


def _var_keys(rng, n: int, prefixes: np.ndarray, lmin: int, lmax: int):
    """Keys = one of the given 8-byte prefixes || random suffix; length U{lmin..lmax}."""
    klens = rng.integers(lmin, lmax + 1, n).astype(np.int64)
    pad = np.zeros((n, ((lmax + 7) // 8) * 8), dtype=np.uint8)
    pad[:, :8] = prefixes[rng.integers(0, prefixes.shape[0], n)]
    suffix = np.frombuffer(rng.bytes(n * (lmax - 8)), dtype=np.uint8).reshape(n, lmax - 8)
    cols = np.arange(8, lmax)
    mask = cols[None, :] < klens[:, None]
    pad[:, 8:lmax] = np.where(mask, suffix, 0)
    return pad, klens


def _sort_unique_var(pad: np.ndarray, klens: np.ndarray):
    """Sort variable keys bytewise (zero padding + length tie-break), drop duplicates."""
    if pad.shape[0] == 0:
        return pad, klens
    words = pad.view(">u8").reshape(pad.shape[0], -1).astype(np.uint64)
    cols = [klens.astype(np.uint64)] + [words[:, j] for j in range(words.shape[1] - 1, -1, -1)]
    order = np.lexsort(cols)
    pad, klens, words = pad[order], klens[order], words[order]
    if pad.shape[0] > 1:
        same = np.all(words[1:] == words[:-1], axis=1) & (klens[1:] == klens[:-1])
        keep = np.concatenate([[True], ~same])
        pad, klens = pad[keep], klens[keep]
    return pad, klens


def _run_from_var(pad, klens, tags, vlens, rng) -> Run:
    n = pad.shape[0]
    koff = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(klens, out=koff[1:])
    mask = np.arange(pad.shape[1])[None, :] < klens[:, None]
    keys = pad[mask]  # row-major: concatenated keys
    vals, voff = _values(rng, vlens)
    return Run(np.ascontiguousarray(keys), koff, tags.astype(_U64), vals, voff)


def _lognormal_vlen(rng, n):
    v = np.rint(np.exp(rng.normal(np.log(256.0), 1.0, n)))
    return np.clip(v, 16, 4096).astype(np.int64)


def _var_level(rng, n_target_bytes: List[int], prefixes, seq_base, p_tomb):
    """One sorted distinct run of variable keys, cut into files by estimated bytes."""
    total = sum(n_target_bytes)
    est = 36 + 8 + 420 + 4
    n = int(total / est * 1.15) + 64
    pad, klens = _var_keys(rng, n, prefixes, 8, 64)
    pad, klens = _sort_unique_var(pad, klens)
    n = pad.shape[0]
    types = (rng.random(n) >= p_tomb).astype(np.uint8)
    vlens = np.where(types == TYPE_VALUE, _lognormal_vlen(rng, n), 0)
    seqs = _seqs(rng, n, seq_base)
    tags = _tags(seqs, types)
    cum = np.cumsum(klens + 8 + vlens + 4)
    runs = []
    start = 0
    acc = 0
    for tb in n_target_bytes:
        acc += tb
        end = int(np.searchsorted(cum, acc, side="left")) + 1
        end = min(max(end, start + 1), n)
        sl = slice(start, end)
        runs.append(_run_from_var(pad[sl], klens[sl], tags[sl], vlens[sl], rng))
        start = end
    return runs


def plain_variable(seed: Optional[int] = None, scale: float = 1.0) -> Job:
    """1 upper + 6 lower tables of ~32 MiB; keys 8-64 B sharing 1,024 8-byte
    prefixes; lognormal values (median 256 B, clipped to [16, 4096]); 10%
    tombstones; 16 KiB blocks, restart interval 16; bottom level; 32 MiB files.
    """
    seed = workload_seed(2) if seed is None else seed
    rng = np.random.default_rng(seed)
    prefixes = np.frombuffer(rng.bytes(1024 * 8), dtype=np.uint8).reshape(1024, 8)
    size = max(4096, int(32 * MiB * scale))
    upper = _var_level(rng, [size], prefixes, 1 << 54, 0.10)
    lower = _var_level(rng, [size] * 6, prefixes, 1 << 52, 0.10)
    return Job(upper + lower, block_size=16384, restart_interval=16, bloom_bits_per_key=10,
               bottommost=1, target_file_size=size, name=f"plain-variable-7x{32 * scale:g}MiB")


# ----------------------------------------------------------------------------
# batch: uneven jobs


def batch_job_sizes(job: int, seed: Optional[int] = None):
    """(n_lower, [upper MiB, lower MiB...]) for batch job `job`."""
    seed = workload_seed(3, job) if seed is None else seed
    rng = np.random.default_rng(seed)
    n_lower = int(rng.integers(1, 13))
    sizes = [int(s) for s in rng.integers(2, 65, n_lower + 1)]
    return n_lower, sizes


def batch_job(job: int, seed: Optional[int] = None, scale: float = 1.0) -> Job:
    """Batch job: 1 upper + U{1..12} lower tables of U{2..64} MiB each; 16-byte
    keys over a per-job salted id space of 2**22; values U{100..1024} B; 5%
    tombstones; 4 KiB blocks; 64 MiB output files; bottom level on even jobs.
    """
    seed = workload_seed(3, job) if seed is None else seed
    n_lower, sizes = batch_job_sizes(job, seed)
    rng = np.random.default_rng(seed ^ 0x5EED)
    salt = int(rng.integers(0, 2**63))
    est = 16 + 8 + 562 + 4
    counts = [max(8, int(s * MiB * scale / est)) for s in sizes]
    vfn = lambda n: rng.integers(100, 1025, n).astype(np.int64)  # noqa: E731
    space = 1 << 22
    up_ids = rng.choice(space, min(counts[0], space), replace=False)
    low_total = min(sum(counts[1:]), space)
    low_ids = rng.choice(space, low_total, replace=False)
    low_counts = counts[1:]
    if sum(low_counts) != low_total:  # only when the id space is exhausted
        low_counts = _split_counts(low_total, n_lower)
    upper = _fixed_level(rng, _sorted_key16(up_ids, salt), [up_ids.shape[0]], 1 << 54, vfn, 0.05)
    lower = _fixed_level(rng, _sorted_key16(low_ids, salt), low_counts, 1 << 52, vfn, 0.05)
    return Job(upper + lower, block_size=4096, restart_interval=16, bloom_bits_per_key=10,
               bottommost=1 if job % 2 == 0 else 0,
               target_file_size=max(1, int(64 * MiB * scale)), name=f"batch-job{job}")


def job_input_bytes_estimate(job: Job) -> int:
    return sum(r.approx_bytes() for r in job.runs)


# ----------------------------------------------------------------------------
# tiny adversarial jobs for tests


def tiny_job(seed: int, n_inputs: int = 3, entries: int = 40, key_alphabet: int = 3,
             key_len: tuple = (1, 3), val_len: tuple = (0, 12), p_tomb: float = 0.3,
             mode: str = "l0", max_versions: int = 3, seq_range: int = 64,
             block_size: int = 64, restart_interval: int = 3, target_file_size: int = 256,
             bottommost: int = 1, bloom_bits_per_key: int = 10) -> Job:
    """Small jobs over a tiny key alphabet, forcing duplicates, shared prefixes,
    multi-version keys inside one table, equal tags across tables and tombstones.

    mode "l0": every table draws over the whole key space (all overlap);
    mode "leveled": tables 1.. split one sorted distinct key set (disjoint).
    """
    rng = np.random.default_rng(seed)
    alphabet = np.arange(key_alphabet, dtype=np.uint8) + np.uint8(0x61)
    if key_alphabet > 2:
        alphabet[-1] = 0  # a zero byte makes "ab" vs "ab\\0" orderings appear
    lmax = key_len[1]

    def draw_keys(n):
        kl = rng.integers(key_len[0], key_len[1] + 1, n).astype(np.int64)
        pad = np.zeros((n, ((max(lmax, 1) + 7) // 8) * 8), dtype=np.uint8)
        sym = alphabet[rng.integers(0, key_alphabet, (n, lmax))]
        mask = np.arange(lmax)[None, :] < kl[:, None]
        pad[:, :lmax] = np.where(mask, sym, 0)
        return pad, kl

    def make_run(pad, kl, versions_max):
        pad, kl = _sort_unique_var(pad, kl)
        n = pad.shape[0]
        reps = rng.integers(1, versions_max + 1, n)
        pad = np.repeat(pad, reps, axis=0)
        kl = np.repeat(kl, reps)
        m = pad.shape[0]
        if m == 0:
            return _run_from_var(pad, kl, np.zeros(0, np.uint64), np.zeros(0, np.int64), rng)
        seqs = rng.integers(0, seq_range, m).astype(np.uint64)
        types = (rng.random(m) >= p_tomb).astype(np.uint8)
        tags = _tags(seqs, types)
        # order: user key asc, tag desc; drop duplicate (key, tag) pairs
        words = pad.view(">u8").reshape(m, -1).astype(np.uint64)
        cols = [~tags, kl.astype(np.uint64)] + [words[:, j] for j in range(words.shape[1] - 1, -1, -1)]
        order = np.lexsort(cols)
        pad, kl, tags, words = pad[order], kl[order], tags[order], words[order]
        if m > 1:
            same = (np.all(words[1:] == words[:-1], axis=1) & (kl[1:] == kl[:-1]) & (tags[1:] == tags[:-1]))
            keep = np.concatenate([[True], ~same])
            pad, kl, tags = pad[keep], kl[keep], tags[keep]
        types = (tags & np.uint64(0xFF)).astype(np.int64)
        vlens = np.where(types == TYPE_VALUE, rng.integers(val_len[0], val_len[1] + 1, tags.shape[0]), 0)
        return _run_from_var(pad, kl, tags, vlens.astype(np.int64), rng)

    runs = []
    if mode == "l0":
        for _ in range(n_inputs):
            pad, kl = draw_keys(entries)
            runs.append(make_run(pad, kl, max_versions))
    elif mode == "leveled":
        pad, kl = draw_keys(entries)
        runs.append(make_run(pad, kl, max_versions))
        pad, kl = draw_keys(entries * max(1, n_inputs - 1))
        pad, kl = _sort_unique_var(pad, kl)
        parts = _split_counts(pad.shape[0], max(1, n_inputs - 1))
        s = 0
        for c in parts:
            if c == 0:
                continue
            runs.append(make_run(pad[s:s + c], kl[s:s + c], max_versions))
            s += c
    else:
        raise ValueError(mode)
    runs = [r for r in runs if r.n > 0]  # a table always holds at least one entry
    return Job(runs, block_size=block_size, restart_interval=restart_interval,
               bloom_bits_per_key=bloom_bits_per_key, bottommost=bottommost,
               target_file_size=target_file_size, name=f"tiny-{mode}-{seed}")


# ----------------------------------------------------------------------------
# compressible variants (block compression, the prototype's future work)


def compressible(job: Job, seed: int = 0, compression: int = 1) -> Job:
    """The same job (keys, tags, value lengths) with values that compress, and
    compression switched on for its input and output tables.

    Even-numbered values repeat a short random pattern (1-12 bytes, from a pool
    of 64), so they hold copies at small offsets; odd-numbered values are
    slices of one 16 KiB random text, so entries of a block share substrings
    at offsets up to a few KiB.  One stretch of 40 consecutive entries in four
    (drawn at random) keeps random values, so some blocks do not compress
    enough and are stored raw.
    """
    rng = np.random.default_rng(seed ^ 0x534E4150)  # "SNAP"
    plen = rng.integers(1, 13, 64)
    pstart = np.concatenate([[0], np.cumsum(plen)[:-1]])
    pbytes = np.frombuffer(rng.bytes(int(plen.sum())), dtype=np.uint8)
    text = np.frombuffer(rng.bytes(16384), dtype=np.uint8)
    runs = []
    for r in job.runs:
        vl = np.diff(r.voff).astype(np.int64)
        n = r.n
        raw = np.repeat(rng.integers(0, 4, n // 40 + 1) == 0, 40)[:n]
        pat = rng.integers(0, 64, n)
        shift = rng.integers(0, 16384, n)
        out = np.empty(int(r.voff[-1]), dtype=np.uint8)
        step = max(1, (8 << 20) // max(1, int(vl.mean()) if n else 1))
        for e0 in range(0, n, step):  # entries in slices of about 8 MiB of values
            e1 = min(n, e0 + step)
            lens = vl[e0:e1]
            tot = int(lens.sum())
            if tot == 0:
                continue
            ent = np.repeat(np.arange(e0, e1), lens)
            pos = np.arange(tot) - np.repeat(r.voff[e0:e1] - r.voff[e0], lens)
            even = (ent % 2) == 0
            b = np.where(even, pbytes[pstart[pat[ent]] + pos % plen[pat[ent]]],
                         text[(shift[ent] + pos) % 16384])
            rnd = raw[ent]
            if rnd.any():
                b[rnd] = np.frombuffer(rng.bytes(int(rnd.sum())), dtype=np.uint8)
            out[int(r.voff[e0]):int(r.voff[e0]) + tot] = b
        runs.append(Run(r.keys, r.koff, r.tags, out, r.voff))
    return Job(runs, block_size=job.block_size, restart_interval=job.restart_interval,
               bloom_bits_per_key=job.bloom_bits_per_key, bottommost=job.bottommost,
               target_file_size=job.target_file_size, name=job.name + "-snappy", meta=dict(job.meta),
               compression=compression)
