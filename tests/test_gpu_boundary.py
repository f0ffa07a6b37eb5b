"""GPU tests of the boundary's bookkeeping through the C-ABI: each output
table's key range, device memory from the caller's allocator, the context's
memory limit, and the served form's refusal, cancellation and retry rules.
Output bytes are compared with the oracle's throughout."""
import pytest

import oracle
import sstcheck
from gpu_util import assert_same_files, ctx, say
from workload import plain_small, batch_job, tiny_job

pytestmark = pytest.mark.gpu


def to_dev(blobs):
    import torch
    return [torch.frombuffer(bytearray(b), dtype=torch.uint8).to("cuda") if len(b) else
            torch.empty(0, dtype=torch.uint8, device="cuda") for b in blobs]


def small_entry_job(seed, entries=60000):
    """Many tiny entries: the working set is several times the input bytes."""
    return tiny_job(seed, n_inputs=3, entries=entries, key_alphabet=255, key_len=(16, 16), val_len=(0, 2),
                    mode="l0", block_size=4096, target_file_size=1 << 20)


def check_key_ranges(files, ranges, label):
    """Each file's reported smallest / largest internal key equals its first /
    last key as decoded by the independent table reader."""
    assert len(files) == len(ranges), label
    for i, (f, (so, sl, lo, ll)) in enumerate(zip(files, ranges)):
        keys = first_last_keys(f)
        assert f[so:so + sl] == keys[0], f"{label}: file {i} smallest key"
        assert f[lo:lo + ll] == keys[1], f"{label}: file {i} largest key"


def first_last_keys(f: bytes):
    """(first internal key of the first data block, key of the last index entry)."""
    ft = f[len(f) - 48:len(f) - 8]
    _, p = sstcheck.varint(ft, 0, 40)
    _, p = sstcheck.varint(ft, p, 40)
    ioff, p = sstcheck.varint(ft, p, 40)
    isize, p = sstcheck.varint(ft, p, 40)
    ic = sstcheck.read_block(f, ioff, isize)
    ients, _ = sstcheck.parse_entries(ic)
    boff, q = sstcheck.varint(ients[0].value, 0, len(ients[0].value))
    bsize, q = sstcheck.varint(ients[0].value, q, len(ients[0].value))
    c = sstcheck.read_block(f, boff, bsize)
    ents, _ = sstcheck.parse_entries(c)
    return ents[0].ikey, ients[-1].ikey


@pytest.mark.parametrize("which", ["plain_small", "tiny-variants"])
def test_file_key_ranges(which):
    jobs = [plain_small()] if which == "plain_small" else [
        tiny_job(300 + s, entries=400, key_alphabet=5, key_len=(1, 30), val_len=(0, 300), block_size=200,
                 target_file_size=1500, restart_interval=3) for s in range(3)]
    for k, job in enumerate(jobs):
        ins = oracle.build_input_tables(job)
        ref = oracle.compact(ins, job.options())
        assert ref.status == 0
        r = ctx().compact(ins, job.options())
        assert_same_files(r.files, ref.files, f"{which}-{k} host")
        check_key_ranges(r.files, r.key_ranges, f"{which}-{k} host")
        rd = ctx().compact_dev(to_dev(ins), job.options())
        files = [t.cpu().numpy().tobytes() for t in rd.files]
        assert_same_files(files, ref.files, f"{which}-{k} device")
        check_key_ranges(files, rd.key_ranges, f"{which}-{k} device")
        say(f"[gpu] key ranges {which}-{k}: {len(files)} files")


def test_torch_allocator_gives_the_same_bytes():
    import torch
    from paper_2004_03054_amd import Context
    job = batch_job(2, scale=1 / 64)
    ins = oracle.build_input_tables(job)
    ref = oracle.compact(ins, job.options())
    c = Context(0)
    try:
        c.use_torch_allocator(True)
        before = torch.cuda.memory_allocated()
        r = c.compact_dev(to_dev(ins), job.options())
        files = [t.cpu().numpy().tobytes() for t in r.files]
        assert_same_files(files, ref.files, "torch allocator")
        during = torch.cuda.memory_allocated()
        held = c.mem_held()
        say(f"[gpu] torch allocator: held {held >> 20} MiB, torch allocated {before >> 20} -> {during >> 20} MiB")
        assert held > 0 and during - before >= held  # the working buffers are torch's
        # outputs kept by the caller also come from torch, and go back to it
        r2 = c.compact_dev(to_dev(ins), job.options(), materialize=False)
        assert r2.status == 0
        c.use_torch_allocator(False)
        assert torch.cuda.memory_allocated() <= during
        r3 = c.compact_dev(to_dev(ins), job.options())
        assert [t.cpu().numpy().tobytes() for t in r3.files] == ref.files
    finally:
        c.close()


def test_memory_limit():
    from paper_2004_03054_amd import Context
    job = plain_small()
    ins = oracle.build_input_tables(job)
    ref = oracle.compact(ins, job.options())
    c = Context(0)
    try:
        c.set_mem_limit(1 << 20)
        r = c.compact_dev(to_dev(ins), job.options())
        assert r.name == "NOMEM", r.name
        assert c.mem_held() <= 1 << 20
        c.set_mem_limit(0)
        r = c.compact_dev(to_dev(ins), job.options())
        assert [t.cpu().numpy().tobytes() for t in r.files] == ref.files
        # the working buffers stay with the context; the output-table buffer
        # went to the result and is needed again by the next call
        need = c.mem_held() + sum(len(t) for t in r.files)
        c.set_mem_limit(need + (1 << 20))
        r = c.compact_dev(to_dev(ins), job.options())
        assert [t.cpu().numpy().tobytes() for t in r.files] == ref.files
        say(f"[gpu] memory limit: job needs {need >> 20} MiB")
    finally:
        c.close()


def test_server_refuses_a_job_over_the_budget():
    from paper_2004_03054_amd import Server
    big = batch_job(8, scale=1 / 16)
    small = [tiny_job(s, mode="l0") for s in range(3)]
    ins_big = oracle.build_input_tables(big)
    ins_small = [oracle.build_input_tables(j) for j in small]
    budget = 3 * sum(map(len, ins_big)) // 2  # below the big job's 3x footprint, above the small ones'
    srv = Server(0, hbm_budget=budget, workers=2)
    try:
        dev_small = [to_dev(i) for i in ins_small]
        tickets = [srv.submit(d, j.options()) for d, j in zip(dev_small, small)]
        with pytest.raises(MemoryError):
            srv.submit(to_dev(ins_big), big.options())
        outs = [srv.poll(t)[0] for t in tickets]
    finally:
        srv.close()
    for k, (r, j, i) in enumerate(zip(outs, small, ins_small)):
        ref = oracle.compact(i, j.options())
        assert r.status == 0
        assert_same_files(r.files, ref.files, f"small job {k} beside a refused job")


def test_server_cancel():
    from paper_2004_03054_amd import Server
    jobs = [batch_job(3, scale=1 / 32)] + [tiny_job(20 + s, mode="leveled") for s in range(5)]
    ins = [oracle.build_input_tables(j) for j in jobs]
    # one worker, one job per pass, a budget for one job at a time: the later
    # jobs wait in the queue while the first runs
    srv = Server(0, hbm_budget=4 * max(sum(map(len, i)) for i in ins) + (2 << 20), max_batch_jobs=1, workers=1)
    try:
        dev = [to_dev(i) for i in ins]
        tickets = [srv.submit(d, j.options()) for d, j in zip(dev, jobs)]
        cancelled = [srv.cancel(t) for t in tickets[3:]]
        outs = [srv.poll(t)[0] for t in tickets]
    finally:
        srv.close()
    say(f"[gpu] cancel: withdrawn {cancelled}")
    for k, (r, j, i) in enumerate(zip(outs, jobs, ins)):
        if k >= 3 and cancelled[k - 3]:
            assert r.name == "CANCELLED" and not r.files, k
            continue
        ref = oracle.compact(i, j.options())
        assert r.status == 0, (k, r.name)
        assert_same_files(r.files, ref.files, f"job {k} beside cancelled jobs")
    assert any(cancelled), "no job was still waiting to be withdrawn"


def test_batch_over_the_memory_limit_runs_each_job_alone():
    """A pass whose jobs together need more device memory than a worker may
    hold fails as a whole (LUDA_NOMEM); the server then runs each job alone,
    and every job gets the oracle's bytes."""
    from paper_2004_03054_amd import Context, Server
    jobs = [small_entry_job(40 + s) for s in range(3)]
    ins = [oracle.build_input_tables(j) for j in jobs]
    # what one job alone, and the three together, hold on the device
    one = Context(0)
    r = one.compact_dev(to_dev(ins[0]), jobs[0].options(), materialize=False)
    assert r.status == 0
    held_one = max(one.mem_held(), 1)
    one.close()
    three = Context(0)
    res = three.compact_batch([(to_dev(i), j.options()) for i, j in zip(ins, jobs)], device_inputs=True,
                              materialize=False)
    assert all(x.status == 0 for x in res)
    held_three = three.mem_held()
    three.close()
    say(f"[gpu] one job holds {held_one >> 20} MiB, three together {held_three >> 20} MiB; "
        f"inputs {[sum(map(len, i)) >> 10 for i in ins]} KiB")
    assert held_three > held_one * 1.3
    limit = (2 * held_one + held_three) // 3
    # the context-level rule: the batch fails as a whole, each job alone fits
    c = Context(0)
    c.set_mem_limit(limit)
    res = c.compact_batch([(to_dev(i), j.options()) for i, j in zip(ins, jobs)], device_inputs=True)
    assert all(x.name == "NOMEM" for x in res), [x.name for x in res]
    for i, j in zip(ins, jobs):
        x = c.compact_dev(to_dev(i), j.options(), materialize=False)
        assert x.status == 0
    c.close()
    # the server: all three admitted into one pass (their footprints fit the
    # budget together), the pass fails, each job runs alone
    fp = sum(3 * sum(map(len, i)) + (1 << 20) for i in ins)
    assert fp <= limit, (fp, limit)
    srv = Server(0, hbm_budget=limit, workers=1)
    try:
        dev = [to_dev(i) for i in ins]
        tickets = [srv.submit(d, j.options()) for d, j in zip(dev, jobs)]
        outs = [srv.poll(t)[0] for t in tickets]
        mem = srv.memory()
    finally:
        srv.close()
    say(f"[gpu] server memory after the retry: {mem}")
    assert mem["held_by_workers"] <= limit
    for k, (x, j, i) in enumerate(zip(outs, jobs, ins)):
        ref = oracle.compact(i, j.options())
        assert x.status == 0, (k, x.name)
        assert_same_files(x.files, ref.files, f"retried job {k}")
