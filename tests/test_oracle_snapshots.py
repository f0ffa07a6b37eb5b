"""Pins of the oracle's drop rule under live snapshots (a reading: the paper
names the drop of stale versions, Sec. II-A, without snapshots).

What a compaction must preserve is what readers see.  A reader at snapshot s
sees, per user key, the newest version with sequence <= s; a reader of the
current state sees the newest version; a deletion reads as absent.  Checked
here, from the entries decoded back out of the output tables, on small jobs
full of multi-version keys and with snapshots placed on and between the
versions' sequence numbers:

* every reader (each snapshot and the current state) reads the same from the
  outputs as from the inputs; below a level that is not the bottom one, lower
  levels may still hold older values of any key, so each key also gets an
  older value underneath on both sides;
* nothing superfluous is kept: every output version is what some reader sees,
  and at the bottom level every output deletion hides an older output value;
* with no snapshots the rule is the plain one (same bytes as without the
  option), and entry counts add up.
"""
import struct

import numpy as np
import pytest

import oracle
from sstcheck import check_output, tag_of, user_key
from workload import tiny_job

CURRENT = 1 << 60


def versions_of(pairs):
    """user key -> [(seq, type, value)] newest first, from (ikey, value) pairs."""
    by = {}
    for ik, v in pairs:
        t = tag_of(ik)
        by.setdefault(user_key(ik), []).append((t >> 8, t & 0xFF, v))
    for k in by:
        by[k].sort(key=lambda x: (-x[0], -x[1]))
    return by


def read(vers, s, older_value):
    """What a reader at snapshot s sees for one key (None: absent)."""
    for seq, typ, v in vers:
        if seq <= s:
            return v if typ == 1 else None
    return older_value


def input_pairs(job):
    out = []
    for r in job.runs:
        for k, tag, v in r.entries():
            out.append((k + struct.pack("<Q", tag), v))
    return out


def check(job, snaps):
    opts = dict(job.options())
    opts["snapshots"] = snaps
    ins = oracle.build_input_tables(job)
    res = oracle.compact(ins, opts)
    assert res.status == 0, res.error
    got = check_output(res.files, opts) if res.files else []
    vin, vout = versions_of(input_pairs(job)), versions_of(got)
    readers = list(snaps) + [CURRENT]
    lower = None if job.bottommost else b"<older value below this level>"
    for k, vi in vin.items():
        vo = vout.get(k, [])
        for s in readers:
            assert read(vi, s, lower) == read(vo, s, lower), (k, s, vi, vo)
        # minimality: each kept version is seen by a reader of the outputs
        seen = set()
        for s in readers:
            for q, (seq, typ, v) in enumerate(vo):
                if seq <= s:
                    seen.add(q)
                    break
        assert seen == set(range(len(vo))), (k, vo, readers)
        if job.bottommost:
            for q, (seq, typ, v) in enumerate(vo):
                if typ == 0:
                    assert any(t == 1 for _, t, _ in vo[q + 1:]), (k, vo)
    assert set(vout) <= set(vin)
    assert res.entries_in == sum(r.n for r in job.runs)
    assert res.entries_in == res.entries_out + res.dropped_shadowed + res.dropped_tombstones
    assert res.entries_out == len(got)
    return res


def snapshot_lists(job, rng, k):
    seqs = sorted({t >> 8 for r in job.runs for _, t, _ in r.entries()})
    cands = set(seqs) | {s + 1 for s in seqs} | {max(0, s - 1) for s in seqs} | {0}
    cands = sorted(cands)
    return sorted(rng.choice(cands, size=min(k, len(cands)), replace=False).tolist())


@pytest.mark.parametrize("seed", range(16))
@pytest.mark.parametrize("bottom", [0, 1])
def test_reads_preserved(seed, bottom):
    job = tiny_job(200 + seed, n_inputs=4, entries=60, key_alphabet=2, key_len=(1, 3), max_versions=5,
                   seq_range=40, p_tomb=0.35, bottommost=bottom, mode="l0")
    rng = np.random.default_rng(seed)
    for k in (1, 2, 5, 12):
        check(job, snapshot_lists(job, rng, k))


def test_no_snapshots_is_the_plain_rule():
    for seed in range(6):
        job = tiny_job(300 + seed, mode="l0", bottommost=seed % 2, max_versions=4)
        ins = oracle.build_input_tables(job)
        plain = oracle.compact(ins, job.options())
        opts = dict(job.options())
        opts["snapshots"] = []
        none = check(job, [])
        assert none.files == plain.files
        # one snapshot below every sequence number sees nothing: the same
        low = oracle.compact(ins, dict(opts, snapshots=[0])) if min(
            t >> 8 for r in job.runs for _, t, _ in r.entries()) > 0 else plain
        assert low.files == plain.files


def test_snapshots_keep_more():
    job = tiny_job(7, n_inputs=4, entries=80, key_alphabet=2, key_len=(1, 2), max_versions=6, seq_range=50,
                   p_tomb=0.2, bottommost=1, mode="l0")
    a = check(job, [])
    b = check(job, [5, 15, 25, 35, 45])
    assert b.entries_out > a.entries_out
    assert b.dropped_shadowed < a.dropped_shadowed


def test_invalid_snapshot_lists():
    job = tiny_job(1)
    ins = oracle.build_input_tables(job)
    for bad in ([5, 5], [9, 3], [1 << 56]):
        assert oracle.compact(ins, dict(job.options(), snapshots=bad)).status == -1
