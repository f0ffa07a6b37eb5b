"""GPU parity of compressed data blocks (block type 1, Snappy streams).

* Inputs written compressed by the oracle are read by the GPU path (their
  streams decoded on the device) and give the oracle's bytes, with outputs
  stored raw and with outputs compressed.
* With compression on, the GPU writer's tables equal the oracle's byte for
  byte: the same streams, the same type per block, the same cuts and
  handles.  Cases span tiny blocks, 4 and 16 KiB blocks (the three plain
  workloads with compressible values), blocks past the decoder's LDS share (global path)
  and past one 64 KiB compression fragment.
* A broken stream gives the oracle's error tuple.
* Each file's smallest and largest internal keys, read from the result,
  equal the first and last keys the independent reader decodes, also when
  the first block is stored compressed.
"""
import pytest

import oracle
import sstcheck
from gpu_util import assert_same_files, ctx, err_tuple, say
from test_oracle_errors import handles, reseal
from test_oracle_snappy import _first_copy
from workload import compressible, plain_small, plain_large, plain_variable, batch_job, tiny_job

pytestmark = pytest.mark.gpu


def to_dev(blobs):
    import torch
    return [torch.frombuffer(bytearray(b), dtype=torch.uint8).to("cuda") for b in blobs]


def first_last(files, opts):
    out = []
    for f in files:
        t = sstcheck.check_table(f, opts["restart_interval"], compression=opts.get("compression", 0))
        out.append((t.blocks[0].entries[0].ikey, t.blocks[-1].entries[-1].ikey))
    return out


def run_both(job, label, out_compression=None, device=False):
    ins = oracle.build_input_tables(job)
    opts = dict(job.options())
    if out_compression is not None:
        opts["compression"] = out_compression
        if not out_compression:
            opts.pop("compression")
    ref = oracle.compact(ins, opts)
    assert ref.status == 0, ref.error
    say(f"[gpu] snappy: {label}: {len(ins)} inputs, {sum(map(len, ins))} bytes, compression {opts.get('compression', 0)}")
    if device:
        res = ctx().compact_dev(to_dev(ins), opts, materialize=lambda t: t.cpu().numpy().tobytes())
    else:
        res = ctx().compact(ins, opts)
    assert res.status == 0, (label, res.name, ctx().last_error())
    assert_same_files(res.files, ref.files, label)
    assert [k for k in res.key_bytes] == first_last(ref.files, opts), label
    return ins, ref


TINY = [
    dict(seed=1, entries=200, val_len=(0, 300), block_size=256, target_file_size=4096),
    dict(seed=2, entries=500, val_len=(0, 2000), block_size=4096, target_file_size=1 << 16, restart_interval=1),
    dict(seed=3, entries=300, val_len=(1000, 5000), block_size=1 << 20, target_file_size=1 << 20),  # > 64 KiB blocks
    dict(seed=4, entries=60, val_len=(0, 12), block_size=64, target_file_size=256, key_alphabet=255,
         key_len=(8, 40)),
]


@pytest.mark.parametrize("k", range(len(TINY)))
def test_tiny_compressed_in_and_out(k):
    kw = dict(TINY[k])
    seed = kw.pop("seed")
    job = compressible(tiny_job(seed, mode=("l0", "leveled")[seed % 2], bottommost=seed % 2, **kw), seed)
    run_both(job, f"tiny {seed}, compressed out")
    run_both(job, f"tiny {seed}, raw out", out_compression=0)


def test_plain_small_compressed():
    job = compressible(plain_small())
    ins, ref = run_both(job, "plain_small", device=True)
    types = [f[b.offset + b.size] for f in ref.files for b in sstcheck.check_table(f, 16, compression=1).blocks]
    assert types.count(1) and types.count(0), "expected both stored forms among the outputs"
    run_both(job, "plain_small, raw out", out_compression=0)


def test_plain_large_scaled_compressed():
    run_both(compressible(plain_large(scale=1 / 16)), "plain_large at 1/16", device=True)


def test_plain_variable_scaled_compressed():
    run_both(compressible(plain_variable(scale=1 / 8)), "plain_variable at 1/8", device=True)


def test_raw_inputs_compressed_outputs():
    job = batch_job(3, scale=1 / 64)
    job.compression = 1  # random values: nearly every block stays raw
    run_both(job, "batch job 3 at 1/64, random values")


def test_batch_mixes_compressed_and_raw_jobs():
    jobs = [compressible(tiny_job(s, entries=300, val_len=(0, 400), block_size=512, target_file_size=8192), s)
            for s in range(3)] + [tiny_job(7, entries=300, val_len=(0, 400), block_size=512)]
    ins = [oracle.build_input_tables(j) for j in jobs]
    res = ctx().compact_batch([(i, j.options()) for i, j in zip(ins, jobs)], device_inputs=False)
    for k, (r, i, j) in enumerate(zip(res, ins, jobs)):
        ref = oracle.compact(i, j.options())
        assert r.status == ref.status == 0
        assert_same_files(r.files, ref.files, f"batch job {k}")


def test_broken_stream_error_tuple():
    job = compressible(plain_small())
    ts = [bytearray(t) for t in oracle.build_input_tables(job)]
    _, hs = handles(bytes(ts[1]))
    k = next(i for i, (bo, bs) in enumerate(hs) if ts[1][bo + bs] == 1 and i > 3)
    bo, bs = hs[k]
    at = _first_copy(bytes(ts[1][bo:bo + bs]))
    kind = ts[1][bo + at] & 3
    if kind == 1:
        ts[1][bo + at] &= 0x1F
        ts[1][bo + at + 1] = 0
    else:
        ts[1][bo + at + 1:bo + at + 1 + (2 if kind == 2 else 4)] = bytes(2 if kind == 2 else 4)
    reseal(ts[1], bo, bs)
    ins = [bytes(t) for t in ts]
    ref = oracle.compact(ins, job.options())
    res = ctx().compact(ins, job.options())
    say(f"[gpu] snappy: broken stream in block {k}: oracle {ref.error}")
    assert ref.status == oracle.STATUS_CODES["CORRUPT_FORMAT"] and ref.error.offset == at
    assert res.status == ref.status and err_tuple(res.error) == err_tuple(ref.error)
