"""GPU parity of the drop rule under live snapshots: the library keeps
exactly the versions the oracle keeps (every output byte compared), alone, in
a batch next to jobs without snapshots, and through the request loop."""
import numpy as np
import pytest

import oracle
from gpu_util import assert_same_files, ctx, say
from workload import plain_small, plain_large, tiny_job

pytestmark = pytest.mark.gpu


def seqs_of(job):
    return sorted({t >> 8 for r in job.runs for _, t, _ in r.entries()})


def snaps_for(job, rng, k):
    """k snapshots on, just above and just below the jobs' sequence numbers."""
    s = seqs_of(job)
    cand = sorted(set(s) | {x + 1 for x in s} | {max(0, x - 1) for x in s})
    return sorted(rng.choice(cand, size=min(k, len(cand)), replace=False).tolist())


def both(job, opts, label, ins=None):
    ins = ins if ins is not None else oracle.build_input_tables(job)
    ref = oracle.compact(ins, opts)
    res = ctx().compact(ins, opts)
    say(f"[gpu] {label}: {len(opts.get('snapshots', []))} snapshots, {ref.entries_out} kept")
    assert res.status == ref.status == 0, (label, res.name, ctx().last_error())
    assert_same_files(res.files, ref.files, label)
    assert (res.entries_out, res.dropped_shadowed, res.dropped_tombstones) == \
        (ref.entries_out, ref.dropped_shadowed, ref.dropped_tombstones), label
    return res, ref


@pytest.mark.parametrize("seed", range(8))
def test_tiny_with_snapshots(seed):
    job = tiny_job(500 + seed, n_inputs=4, entries=60, key_alphabet=2, key_len=(1, 3), max_versions=5,
                   seq_range=40, p_tomb=0.35, bottommost=seed % 2, mode="l0")
    rng = np.random.default_rng(seed)
    for k in (1, 3, 12):
        opts = dict(job.options(), snapshots=snaps_for(job, rng, k))
        both(job, opts, f"tiny{seed}-k{k}")


def test_plain_small_with_snapshots():
    job = plain_small()
    s = seqs_of(job)
    opts = dict(job.options(), snapshots=[s[len(s) // 5], s[len(s) // 2], s[-2]])
    both(job, opts, "plain_small-snaps")


def test_plain_large_scaled_with_snapshots():
    job = plain_large(scale=1 / 64)
    s = seqs_of(job)
    opts = dict(job.options(), snapshots=[s[k * len(s) // 9] for k in range(1, 9)])
    both(job, opts, "plain_large-x1/64-snaps")


def test_batch_mixes_snapshot_rules():
    jobs = [tiny_job(600 + k, n_inputs=3, entries=50, key_alphabet=2, key_len=(1, 2), max_versions=4,
                     seq_range=30, p_tomb=0.3, bottommost=k % 2, mode="l0") for k in range(6)]
    rng = np.random.default_rng(3)
    optss = [dict(j.options(), snapshots=snaps_for(j, rng, 4)) if k % 2 == 0 else j.options()
             for k, j in enumerate(jobs)]
    ins = [oracle.build_input_tables(j) for j in jobs]
    out = ctx().compact_batch(list(zip(ins, optss)), device_inputs=False)
    for k, (i, o, r) in enumerate(zip(ins, optss, out)):
        ref = oracle.compact(i, o)
        assert r.status == 0, (k, r.name)
        assert_same_files(r.files, ref.files, f"batch job {k}")


def test_served_copies_the_snapshot_list():
    from paper_2004_03054_amd import Server
    import torch
    job = tiny_job(700, n_inputs=4, entries=60, key_alphabet=2, key_len=(1, 3), max_versions=5, seq_range=40,
                   p_tomb=0.35, bottommost=1, mode="l0")
    ins = oracle.build_input_tables(job)
    opts = dict(job.options(), snapshots=snaps_for(job, np.random.default_rng(9), 5))
    ref = oracle.compact(ins, opts)
    srv = Server(0, hbm_budget=1 << 30, max_batch_jobs=0, workers=1)
    try:
        dev = [torch.frombuffer(bytearray(b), dtype=torch.uint8).to("cuda") for b in ins]
        t = srv.submit(dev, opts)  # the option arrays are gone once submit returns
        r, _ = srv.poll(t)
    finally:
        srv.close()
    assert r.status == 0, r.name
    assert_same_files(r.files, ref.files, "served with snapshots")


def test_invalid_snapshot_lists():
    job = tiny_job(1)
    ins = oracle.build_input_tables(job)
    for bad in ([5, 5], [9, 3], [1 << 56]):
        r = ctx().compact(ins, dict(job.options(), snapshots=bad))
        assert r.status == -1, (bad, r.status)
