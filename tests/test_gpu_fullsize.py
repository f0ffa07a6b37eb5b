"""GPU parity at the stated sizes of the batch and served workloads.

* One batched pass (luda_compact_batch, device inputs) over the first jobs of
  the 256-job batch workload at full size, until their input exceeds 4.5 GiB,
  so that output offsets inside the pass pass 2^32.  Every job's output
  tables are compared with the oracle's by length and SHA-256.
* A served run of 7 full-size jobs of the same mixture, 2 workers, under a
  budget that admits about two jobs at a time; half of the later requests
  read an earlier request's output tables (left in HBM) as their first lower
  input.  Each job is compared with the oracle and with itself run alone.

Inputs come from the oracle's table writer; the oracle runs on a host thread
pool (its C code runs without the interpreter lock).
"""
import hashlib
import os
from concurrent.futures import ThreadPoolExecutor

import pytest

import oracle
from gpu_util import say
from workload import batch_job

pytestmark = pytest.mark.gpu

BATCH_MIN_BYTES = int(4.5 * 2**30)
THREADS = min(16, os.cpu_count() or 1)


def digest(files):
    return [(len(f), hashlib.sha256(f).hexdigest()) for f in files]


def dev_digest(tensors):
    return digest([t.cpu().numpy().tobytes() for t in tensors])


def prepare(j):
    """Job j of the batch workload at full size: input tables, the oracle's
    result as digests (the output bytes themselves are not kept)."""
    job = batch_job(j)
    ins = oracle.build_input_tables(job)
    ref = oracle.compact(ins, job.options())
    meta = (job.name, job.options())  # the generated entries themselves are dropped
    del job
    return meta, ins, ref.status, digest(ref.files), (ref.entries_in, ref.entries_out)


def to_dev(blobs):
    import torch
    return [torch.frombuffer(bytearray(b), dtype=torch.uint8).to("cuda") for b in blobs]


def test_batch_workload_full_size_one_pass():
    import torch
    from paper_2004_03054_amd import Context
    jobs, total, j = [], 0, 0
    with ThreadPoolExecutor(max_workers=THREADS) as ex:
        while total <= BATCH_MIN_BYTES:
            futs = [ex.submit(prepare, j + k) for k in range(THREADS)]
            for f in futs:
                meta, ins, st, dg, counts = f.result()
                if total > BATCH_MIN_BYTES:
                    break
                dev = to_dev(ins)
                total += sum(map(len, ins))
                jobs.append((meta, dev, st, dg, counts))
                del ins
            j += THREADS
            say(f"[gpu] batch workload: {len(jobs)} jobs prepared, {total / 2**30:.2f} GiB")
    say(f"[gpu] one batched pass over {len(jobs)} full-size jobs, {total / 2**30:.2f} GiB of input")
    c = Context(0)
    try:
        res = c.compact_batch([(d, meta[1]) for meta, d, *_ in jobs], device_inputs=True, materialize=False)
        assert all(r.status == 0 for r in res), [r.name for r in res]
        out_bytes = sum(r.bytes_out for r in res)
        say(f"[gpu] batched pass: {out_bytes / 2**30:.2f} GiB of output tables")
        assert out_bytes > 2**32, "the pass's output offsets should pass 2^32"
        del res
        res = c.compact_batch([(d, meta[1]) for meta, d, *_ in jobs], device_inputs=True,
                              materialize=lambda t: t.clone())
        for k, (r, (meta, _d, st, dg, counts)) in enumerate(zip(res, jobs)):
            assert r.status == st == 0, (k, r.name)
            assert (r.entries_in, r.entries_out) == counts, k
            assert dev_digest(r.files) == dg, f"job {k} ({meta[0]}): output differs from the oracle's"
            r.files = None
        torch.cuda.synchronize()
    finally:
        c.close()


def test_served_workload_full_size():
    import torch
    from paper_2004_03054_amd import Context, Server
    picks = [8, 18, 2, 14, 12, 21, 15]  # jobs of 1-4 lower tables: about 100-250 MiB each
    with ThreadPoolExecutor(max_workers=THREADS) as ex:
        prepared = list(ex.map(prepare, picks))
    sizes = [sum(map(len, p[1])) for p in prepared]
    # about two jobs' footprints (3x input + 1 MiB) at once: later jobs wait for budget
    budget = 2 * (3 * max(sizes) + (1 << 20)) + (64 << 20)
    say(f"[gpu] served: {len(picks)} jobs of {[s >> 20 for s in sizes]} MiB, budget {budget >> 20} MiB")
    dev = [to_dev(p[1]) for p in prepared]
    srv = Server(0, hbm_budget=budget, workers=2, max_batch_jobs=0, host_outputs=False)
    try:
        first = [srv.submit(dev[k], prepared[k][0][1]) for k in range(4)]
        outs = [srv.poll(t, materialize=lambda t: t.clone()) for t in first]
        # later requests: jobs 4..6, two of them reading an earlier request's
        # output tables (in HBM) in place of their first lower table
        reuse = {4: 0, 6: 2}
        later_inputs = []
        for k in range(4, len(picks)):
            ins = dev[k]
            if k in reuse:
                ins = [ins[0]] + list(outs[reuse[k]][0].files) + list(ins[2:])
            later_inputs.append(ins)
        later = [srv.submit(ins, prepared[k][0][1]) for k, ins in zip(range(4, len(picks)), later_inputs)]
        outs += [srv.poll(t, materialize=lambda t: t.clone()) for t in later]
        st = srv.stats()
        mem = srv.memory()
    finally:
        srv.close()
    say(f"[gpu] served stats {st}, memory {mem}")
    assert st["jobs"] == len(picks)
    assert mem["held_by_workers"] <= budget
    c = Context(0)
    try:
        for k in range(len(picks)):
            r, lat = outs[k]
            opts = prepared[k][0][1]
            assert r.status == 0, (k, r.name)
            if k < 4 or k == 5:
                ref_dg = prepared[k][3]
                ins_dev = dev[k]
            else:  # the oracle on the same inputs, earlier outputs included
                ins_dev = later_inputs[k - 4]
                host = [t.cpu().numpy().tobytes() for t in ins_dev]
                ref = oracle.compact(host, opts)
                assert ref.status == 0
                ref_dg = digest(ref.files)
            assert dev_digest(r.files) == ref_dg, f"served job {k}: output differs from the oracle's"
            alone = c.compact_dev(ins_dev, opts, materialize=lambda t: t.clone())
            assert dev_digest(alone.files) == ref_dg, f"served job {k}: alone vs in the mix"
            say(f"[gpu] served job {k}: {len(r.files)} files, latency {lat:.1f} ms, identical")
        torch.cuda.synchronize()
    finally:
        c.close()
