"""Pins of the oracle's merge, drop and pack semantics.

* brute-force replay: for every user key the newest version wins (largest
  tag; on equal tags the earlier input, then the earlier position), and a
  winning deletion disappears at the bottom level -- checked against the
  entries decoded back out of the oracle's output tables;
* closed form for the survivor count;
* the independent table checker (own CRC, xxhash-package Bloom probes) on every
  output table: layout, restart pattern, index keys, filters, cut rules.
"""
import struct

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st, HealthCheck

import oracle
from sstcheck import check_output
from workload import tiny_job, plain_small, plain_large, plain_variable, batch_job


def replay(job):
    best = {}
    for i, r in enumerate(job.runs):
        for p, (k, tag, v) in enumerate(r.entries()):
            cand = (tag, -i, -p)
            if k not in best or cand > best[k][0]:
                best[k] = (cand, tag, v)
    out = []
    for k in sorted(best):
        _, tag, v = best[k]
        if job.bottommost and (tag & 0xFF) == 0:
            continue
        out.append((k + struct.pack("<Q", tag), v))
    return out


def check_job(job):
    ins = oracle.build_input_tables(job)
    res = oracle.compact(ins, job.options())
    assert res.status == 0, res.error
    got = check_output(res.files, job.options()) if res.files else []
    exp = replay(job)
    assert got == exp
    # closed form
    newest = {}
    for i, r in enumerate(job.runs):
        for k, tag, _ in r.entries():
            newest[k] = max(newest.get(k, -1), tag)
    n_del = sum(1 for t in newest.values() if (t & 0xFF) == 0)
    assert res.entries_out == len(newest) - (n_del if job.bottommost else 0)
    assert res.entries_in == sum(r.n for r in job.runs)
    assert res.entries_in == res.entries_out + res.dropped_shadowed + res.dropped_tombstones
    return res


@pytest.mark.parametrize("seed", range(12))
@pytest.mark.parametrize("mode", ["l0", "leveled"])
def test_replay_tiny(seed, mode):
    check_job(tiny_job(seed, mode=mode, bottommost=seed % 2))


@settings(max_examples=60, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(seed=st.integers(0, 2**31), n_inputs=st.integers(1, 5), entries=st.integers(0, 40),
       alphabet=st.integers(1, 4), klen=st.integers(1, 4), vmax=st.integers(0, 40),
       block=st.integers(1, 200), R=st.integers(1, 5), target=st.integers(1, 600),
       bottom=st.integers(0, 1), mode=st.sampled_from(["l0", "leveled"]),
       p_tomb=st.floats(0, 1), bpk=st.integers(1, 20))
def test_replay_hypothesis(seed, n_inputs, entries, alphabet, klen, vmax, block, R, target, bottom,
                           mode, p_tomb, bpk):
    job = tiny_job(seed, n_inputs=n_inputs, entries=entries, key_alphabet=alphabet,
                   key_len=(1, klen), val_len=(0, vmax), p_tomb=p_tomb, mode=mode,
                   block_size=block, restart_interval=R, target_file_size=target,
                   bottommost=bottom, bloom_bits_per_key=bpk)
    check_job(job)


def test_zero_inputs_and_all_dropped():
    res = oracle.compact([], dict(block_size=4096, restart_interval=16, bloom_bits_per_key=10,
                                  bottommost=1, target_file_size=1 << 20))
    assert res.status == 0 and res.files == [] and res.entries_in == 0
    # every entry a deletion at the bottom level: no output file at all
    job = tiny_job(3, p_tomb=1.0, bottommost=1)
    res = check_job(job)
    assert res.files == [] and res.entries_out == 0


def test_plain_small_shape():
    job = plain_small()
    res = check_job_fast(job)
    assert res.entries_in == 30000
    assert 100 < res.dropped_shadowed < 300
    assert len(res.files) == 2


def check_job_fast(job):
    """Like check_job but with a vectorised replay (for the larger workloads)."""
    ins = oracle.build_input_tables(job)
    res = oracle.compact(ins, job.options())
    assert res.status == 0, res.error
    got = check_output(res.files, job.options())
    # replay via numpy: newest version per key
    keys, tags, src = [], [], []
    for i, r in enumerate(job.runs):
        for p in range(r.n):
            keys.append(r.key(p))
        tags.append(r.tags)
        src.extend((i, p) for p in range(r.n))
    tags = np.concatenate(tags)
    best = {}
    for idx, k in enumerate(keys):
        t = int(tags[idx])
        cand = (t, -src[idx][0], -src[idx][1])
        if k not in best or cand > best[k][0]:
            best[k] = (cand, idx)
    exp_keys = []
    for k in sorted(best):
        idx = best[k][1]
        t = int(tags[idx])
        if job.bottommost and (t & 0xFF) == 0:
            continue
        exp_keys.append(k + struct.pack("<Q", t))
    assert [g[0] for g in got] == exp_keys
    return res


@pytest.mark.parametrize("make", [lambda: plain_large(scale=1 / 256), lambda: plain_variable(scale=1 / 256),
                                  lambda: batch_job(0, scale=1 / 256), lambda: batch_job(1, scale=1 / 256)])
def test_scaled_workloads(make):
    check_job_fast(make())
