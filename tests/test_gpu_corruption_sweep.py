"""Seeded corruption sweep: random byte edits in the footer, index block and
data blocks of small tables (plain and compressed), each compacted by the GPU
path and by the oracle.  The first-error tuple (status, input, where, phase,
block, offset) must agree, and when both succeed (an edit in a region the
compaction never reads, such as the filter block) the output tables must be
the same bytes.  Half of the edits inside a block are followed by a fresh
trailer checksum, so that checks past the checksum are reached too."""
import numpy as np
import pytest

import oracle
from gpu_util import assert_same_files, ctx, err_tuple, say
from test_oracle_errors import handles, reseal
from workload import compressible, tiny_job

pytestmark = pytest.mark.gpu

CASES = 240


def _inputs(seed):
    job = tiny_job(seed, n_inputs=3, entries=80, key_alphabet=5, key_len=(2, 6), val_len=(0, 40), p_tomb=0.2,
                   mode=("l0", "leveled")[seed % 2], block_size=160, restart_interval=(3, 1, 16)[seed % 3])
    if seed % 4 == 3:
        job = compressible(job, seed)
    return job, [bytearray(t) for t in oracle.build_input_tables(job)]


def _edit(rng, t: bytearray):
    """One random edit; returns a label."""
    (io, isz), hs = handles(bytes(t))
    region = rng.integers(0, 4)
    if region == 0:  # footer
        p = len(t) - 48 + int(rng.integers(0, 48))
        t[p] ^= int(rng.integers(1, 256))
        return f"footer +{p - (len(t) - 48)}"
    if region == 1:  # index block (contents or trailer)
        p = io + int(rng.integers(0, isz + 5))
        t[p] ^= int(rng.integers(1, 256))
        if rng.integers(0, 2) and p < io + isz:
            reseal(t, io, isz)
            return f"index +{p - io} resealed"
        return f"index +{p - io}"
    # a data block: contents, type byte or checksum
    k = int(rng.integers(0, len(hs)))
    bo, bs = hs[k]
    p = bo + int(rng.integers(0, bs + 5))
    t[p] ^= int(rng.integers(1, 256))
    if rng.integers(0, 2) and p <= bo + bs:
        reseal(t, bo, bs)
        return f"block {k} +{p - bo} resealed"
    return f"block {k} +{p - bo}"


def test_random_edits_match_the_oracle():
    rng = np.random.default_rng(20261203)
    c = ctx()
    kinds = {}
    for case in range(CASES):
        seed = int(rng.integers(0, 1 << 30))
        job, ts = _inputs(seed)
        which = int(rng.integers(0, len(ts)))
        label = _edit(rng, ts[which])
        ins = [bytes(t) for t in ts]
        ref = oracle.compact(ins, job.options())
        got = c.compact(ins, job.options())
        tag = f"case {case} (seed {seed}, input {which}, {label})"
        assert got.status == ref.status, (tag, got.name, ref.error, c.last_error())
        if ref.status:
            assert err_tuple(got.error) == err_tuple(ref.error), (tag, got.error, ref.error)
        else:
            assert_same_files(got.files, ref.files, tag)
        kinds[oracle.STATUS_NAMES[ref.status]] = kinds.get(oracle.STATUS_NAMES[ref.status], 0) + 1
    say(f"[gpu] corruption sweep: {CASES} cases, outcomes {kinds}")
    assert len(kinds) >= 3  # the sweep reaches several kinds of outcome
