"""luda_compact_dev_noalloc: the compaction without device allocations.

Its working buffers come from the library's static scratch memory and its
output tables go into a buffer the caller passes.  Two calls in a row (the
second on a smaller job) must give the same bytes as luda_compact_dev, the
existing entry point, and as the oracle; sizes past either limit fail with
LUDA_NOMEM and a message naming it.
"""
import pytest

import oracle
from gpu_util import say
from workload import plain_small, tiny_job

pytestmark = pytest.mark.gpu

SCRATCH_BYTES = 256 << 20  # LUDA_SCRATCH_BYTES in include/luda.h


def to_dev(blobs):
    import torch
    return [torch.frombuffer(bytearray(b), dtype=torch.uint8).to("cuda") for b in blobs]


def host(tensors):
    return [t.cpu().numpy().tobytes() for t in tensors]


def test_noalloc_matches_compact_dev_on_two_calls():
    import torch
    from paper_2004_03054_amd import Context
    jobs = [plain_small(), tiny_job(5, mode="l0", bottommost=0)]  # the second is smaller
    c = Context(0)
    try:
        out = torch.empty(16 << 20, dtype=torch.uint8, device="cuda")
        for job in jobs:
            ins = oracle.build_input_tables(job)
            ref = oracle.compact(ins, job.options())
            assert ref.status == 0
            dev = to_dev(ins)
            say(f"[gpu] no-alloc call: {job.name}, {sum(map(len, ins))} input bytes")
            want = c.compact_dev(dev, job.options())
            assert want.status == 0, want.name
            got = c.compact_dev_noalloc(dev, job.options(), out, materialize=lambda t: t.clone())
            assert got.status == 0, (got.name, c.last_error())
            assert host(got.files) == host(want.files) == ref.files, job.name
            assert (got.entries_in, got.entries_out) == (want.entries_in, want.entries_out)
            assert got.key_ranges == want.key_ranges
            used = c.counters().get("scratch_bytes_used", 0)
            assert 0 < used <= SCRATCH_BYTES
            say(f"[gpu] {job.name}: {len(got.files)} files identical, scratch used {int(used)} bytes")
        torch.cuda.synchronize()
    finally:
        c.close()


def test_noalloc_rejects_sizes_past_its_limits():
    import torch
    from paper_2004_03054_amd import Context
    c = Context(0)
    try:
        job = plain_small()
        ins = oracle.build_input_tables(job)
        dev = to_dev(ins)
        small_out = torch.empty(4096, dtype=torch.uint8, device="cuda")
        r = c.compact_dev_noalloc(dev, job.options(), small_out)
        assert r.name == "NOMEM" and "output buffer" in c.last_error(), (r.name, c.last_error())
        # many tiny entries: the working buffers exceed the scratch memory
        big = tiny_job(9, n_inputs=3, entries=400000, key_alphabet=255, key_len=(16, 16), val_len=(0, 2),
                       mode="l0", block_size=4096, target_file_size=1 << 20)
        big_ins = oracle.build_input_tables(big)
        say(f"[gpu] no-alloc over the scratch limit: {sum(map(len, big_ins))} input bytes")
        out = torch.empty(2 * sum(map(len, big_ins)) + (1 << 20), dtype=torch.uint8, device="cuda")
        r = c.compact_dev_noalloc(to_dev(big_ins), big.options(), out)
        assert r.name == "NOMEM" and "scratch" in c.last_error(), (r.name, c.last_error())
        # the entry point still works afterwards, and agrees with the oracle
        out = torch.empty(16 << 20, dtype=torch.uint8, device="cuda")
        r = c.compact_dev_noalloc(dev, job.options(), out, materialize=lambda t: t.clone())
        assert r.status == 0 and host(r.files) == oracle.compact(ins, job.options()).files
        torch.cuda.synchronize()
    finally:
        c.close()
