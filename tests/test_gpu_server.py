"""GPU parity of the served form (luda_server_* through the C-ABI): jobs
submitted together, admitted under a memory budget and run in batched passes
by two workers, give each job exactly the oracle's output bytes, the same
as when it runs alone."""
import pytest

import oracle
from gpu_util import assert_same_files, ctx, err_tuple, say
from workload import plain_small, batch_job, tiny_job

pytestmark = pytest.mark.gpu


def to_dev(blobs):
    import torch
    return [torch.frombuffer(bytearray(b), dtype=torch.uint8).to("cuda") if len(b) else
            torch.empty(0, dtype=torch.uint8, device="cuda") for b in blobs]


def corrupt(blob: bytes, at: int) -> bytes:
    b = bytearray(blob)
    b[at] ^= 0x40
    return bytes(b)


@pytest.mark.parametrize("budget,workers,max_batch", [("1GiB", 2, 0), ("tight", 2, 3), ("tight", 1, 1)])
def test_served_mix_matches_oracle(budget, workers, max_batch):
    from paper_2004_03054_amd import Server
    jobs = [tiny_job(s, mode=("l0", "leveled")[s % 2], bottommost=s % 2) for s in range(8)]
    jobs += [batch_job(4, scale=1 / 64), plain_small(), batch_job(5, scale=1 / 128)]
    ins = [oracle.build_input_tables(j) for j in jobs]
    # one job with a corrupted data block: only it fails
    bad = 3
    ins[bad] = [corrupt(ins[bad][0], 7)] + ins[bad][1:]
    # "tight": twice the largest job's expected footprint (3x its input + 1 MiB),
    # so that only a few jobs are admitted at a time and the rest wait
    fp = max(3 * sum(map(len, i)) + (1 << 20) for i in ins)
    budget_bytes = 1 << 30 if budget == "1GiB" else 2 * fp
    say(f"[gpu] server: {len(jobs)} jobs, budget {budget_bytes >> 20} MiB, {workers} workers, max batch {max_batch}")
    srv = Server(0, hbm_budget=budget_bytes, max_batch_jobs=max_batch, workers=workers)
    try:
        dev = [to_dev(i) for i in ins]
        tickets = [srv.submit(d, j.options()) for d, j in zip(dev, jobs)]
        outs = [srv.poll(t) for t in tickets]
        st = srv.stats()
    finally:
        srv.close()
    say(f"[gpu] server stats {st}")
    assert st["jobs"] == len(jobs)
    for k, ((r, lat), j, i) in enumerate(zip(outs, jobs, ins)):
        ref = oracle.compact(i, j.options())
        assert r.status == ref.status, (k, r.name, str(ref.error))
        if ref.status != 0:
            assert err_tuple(r.error) == err_tuple(ref.error), (k, r.error, ref.error)
            continue
        assert lat >= 0.0
        assert_same_files(r.files, ref.files, f"served job {k}")
        alone = ctx().compact(i, j.options())
        assert alone.files == r.files, f"served job {k}: alone vs mix"


def test_pin_reserve_grows_by_segments():
    from paper_2004_03054_amd import pin_reserve
    before = pin_reserve(0)
    after = pin_reserve(before + (1 << 30))
    say(f"[gpu] pinned pool {before >> 20} -> {after >> 20} MiB")
    assert after >= before + (1 << 30) and after % (1 << 30) == 0
    assert pin_reserve(0) == after  # kept until the process ends
