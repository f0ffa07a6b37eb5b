"""GPU parity: output tables byte-identical to the oracle's, through the C-ABI.

Inputs are written by the oracle's table writer from seeded workloads; the
GPU library compacts them and every output byte is compared with the
oracle's compaction of the same inputs.
"""
import os

import numpy as np
import pytest

import oracle
from gpu_util import assert_same_files, ctx, err_tuple, say
from workload import plain_small, plain_large, plain_variable, batch_job, tiny_job

pytestmark = pytest.mark.gpu


def to_dev(blobs):
    import torch
    return [torch.frombuffer(bytearray(b), dtype=torch.uint8).to("cuda") if len(b) else
            torch.empty(0, dtype=torch.uint8, device="cuda") for b in blobs]


def run_both(job, label, device=False, inputs=None):
    ins = inputs if inputs is not None else oracle.build_input_tables(job)
    say(f"[gpu] {label}: {len(ins)} inputs, {sum(map(len, ins))} bytes")
    ref = oracle.compact(ins, job.options())
    if device:
        res = ctx().compact_dev(to_dev(ins), job.options())
        files = [t.cpu().numpy().tobytes() for t in res.files]
    else:
        res = ctx().compact(ins, job.options())
        files = res.files
    assert res.status == ref.status, (label, res.name, ctx().last_error(), str(ref.error), res.error)
    if ref.status != 0:
        assert err_tuple(res.error) == err_tuple(ref.error), (label, res.error, ref.error)
        return res, ref
    assert_same_files(files, ref.files, label)
    assert (res.entries_in, res.entries_out, res.dropped_shadowed, res.dropped_tombstones) == \
        (ref.entries_in, ref.entries_out, ref.dropped_shadowed, ref.dropped_tombstones), label
    return res, ref


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("mode", ["l0", "leveled"])
def test_tiny(seed, mode):
    run_both(tiny_job(seed, mode=mode, bottommost=seed % 2), f"tiny-{mode}-{seed}")


TINY_VARIANTS = [
    dict(restart_interval=1, block_size=32),
    dict(restart_interval=16, block_size=4096, target_file_size=1 << 20),
    dict(key_len=(1, 40), key_alphabet=2, val_len=(0, 300), block_size=256, restart_interval=4),
    dict(key_len=(17, 33), key_alphabet=2, val_len=(0, 10), entries=200, block_size=512),
    dict(n_inputs=9, entries=30, mode="leveled", block_size=100, target_file_size=300),
    dict(n_inputs=6, entries=80, p_tomb=0.6, bottommost=1, block_size=1, target_file_size=1),
    dict(entries=300, key_alphabet=4, key_len=(3, 6), val_len=(100, 200), block_size=4096, target_file_size=4096,
         restart_interval=7, bloom_bits_per_key=3),
    # many tiny entries per block: the encoder stages a block's entries in
    # several windows; restart arrays of one slot per entry, and of one slot
    dict(entries=1500, key_alphabet=6, key_len=(2, 8), val_len=(0, 4), block_size=65536, restart_interval=1,
         target_file_size=1 << 20),
    dict(entries=1500, key_alphabet=6, key_len=(2, 8), val_len=(0, 40), block_size=65536, restart_interval=500,
         target_file_size=1 << 20),
    # one entry per block, blocks of 20 B to 2.3 KiB: the data block checksum
    # runs over one to five 512-byte rounds, the message start at many
    # offsets of its round (below and above a chunk edge, in the top round
    # and in the one after it)
    dict(entries=1200, key_alphabet=5, key_len=(4, 12), val_len=(0, 2300), block_size=1, restart_interval=1,
         target_file_size=4 << 20),
    # blocks larger than the encoder's LDS stage (encoded from registers)
    dict(entries=150, key_alphabet=5, key_len=(4, 12), val_len=(1500, 5000), block_size=1 << 20, restart_interval=16,
         target_file_size=4 << 20),
]


@pytest.mark.parametrize("vi", range(len(TINY_VARIANTS)))
def test_tiny_variants(vi):
    kw = dict(TINY_VARIANTS[vi])
    for seed in range(3):
        run_both(tiny_job(100 + seed, **kw), f"variant{vi}-{seed}")


def test_long_index_blocks():
    """Index blocks of about 3 MB (hundreds of 4 KiB checksum segments, so the
    segment join folds several segments per lane), in the inputs and in the
    outputs."""
    job = tiny_job(7, n_inputs=2, entries=150000, key_alphabet=20, key_len=(6, 10), val_len=(0, 6), block_size=40,
                   restart_interval=4, target_file_size=4 << 20, mode="leveled", max_versions=2)
    run_both(job, "long-index")
    ins = oracle.build_input_tables(job)
    bad = bytearray(ins[1])
    bad[len(bad) - 48 - 5 - 1000000] ^= 0x01  # a byte inside the second input's index block
    res, ref = run_both(job, "long-index-corrupt", inputs=[ins[0], bytes(bad)])
    assert ref.status != 0


def test_empty_and_all_dropped():
    res = ctx().compact([], dict(block_size=4096, restart_interval=16, bloom_bits_per_key=10, bottommost=1,
                                 target_file_size=1 << 20))
    assert res.status == 0 and res.files == []
    res, ref = run_both(tiny_job(3, p_tomb=1.0, bottommost=1), "all-dropped")
    assert res.files == [] and ref.files == []


def test_plain_small():
    run_both(plain_small(), "plain_small")


def test_plain_small_device_inputs():
    run_both(plain_small(), "plain_small-dev", device=True)


@pytest.mark.parametrize("scale", [1 / 64, 1 / 16])
def test_plain_large_scaled(scale):
    run_both(plain_large(scale=scale), f"plain_large-x{scale}")


@pytest.mark.parametrize("scale", [1 / 64, 1 / 16])
def test_plain_variable_scaled(scale):
    run_both(plain_variable(scale=scale), f"plain_variable-x{scale}")


@pytest.mark.parametrize("job", [0, 1, 7])
def test_batch_jobs_scaled(job):
    run_both(batch_job(job, scale=1 / 32), f"batch-job{job}")


def test_batch_matches_alone():
    jobs = [tiny_job(s, mode=("l0", "leveled")[s % 2], bottommost=s % 2) for s in range(10)]
    jobs += [batch_job(2, scale=1 / 64), plain_small()]
    ins = [oracle.build_input_tables(j) for j in jobs]
    say(f"[gpu] batch of {len(jobs)} jobs")
    out = ctx().compact_batch([(i, j.options()) for i, j in zip(ins, jobs)], device_inputs=False)
    for k, (j, i, r) in enumerate(zip(jobs, ins, out)):
        ref = oracle.compact(i, j.options())
        assert r.status == 0, (k, r.name, ctx().last_error())
        assert_same_files(r.files, ref.files, f"batch job {k}")
        alone = ctx().compact(i, j.options())
        assert alone.files == r.files, f"batch job {k}: alone vs batch"


# full sizes of the benchmark-class workloads: every output byte compared
@pytest.mark.parametrize("make,label", [(lambda: plain_large(), "plain_large-full"), (lambda: plain_variable(), "plain_variable-full")])
def test_full_size(make, label):
    res, ref = run_both(make(), label, device=True)
    say(f"[gpu] {label}: {len(ref.files)} files, {res.entries_in} entries in, {res.entries_out} out")


def test_launch_params_do_not_change_bytes():
    """Every launch setting the autotuner may pick gives the same outputs."""
    job = batch_job(6, scale=1 / 64)
    ins = oracle.build_input_tables(job)
    ref = oracle.compact(ins, job.options())
    c = ctx()
    saved = c.params()
    try:
        for cw, ew, sb in [(4, 2, 1), (16, 4, 64), (8, 16, 4), (16, 16, 32)]:
            c.set_params(cw, ew, sb)
            res = c.compact(ins, job.options())
            assert res.status == 0, (cw, ew, sb, res.name)
            assert_same_files(res.files, ref.files, f"params {cw}/{ew}/{sb}")
        best, ms = c.autotune([(ins, job.options())], device_inputs=False, rounds=1)
        say(f"[gpu] autotune picked {best} ({ms:.2f} ms)")
        res = c.compact(ins, job.options())
        assert_same_files(res.files, ref.files, "autotuned")
    finally:
        c.set_params(**saved)


def test_host_sort_gives_the_same_bytes():
    """The cooperative sort (entries ordered on the host) gives the oracle's
    bytes, alone and in a batch."""
    c = ctx()
    c.set_host_sort(True)
    try:
        for seed in range(4):
            run_both(tiny_job(seed, mode=("l0", "leveled")[seed % 2], bottommost=seed % 2), f"hostsort-tiny-{seed}")
        run_both(plain_small(), "hostsort-plain_small")
        run_both(plain_large(scale=1 / 64), "hostsort-plain_large-x1/64")
        jobs = [tiny_job(20 + s, bottommost=s % 2) for s in range(5)] + [batch_job(3, scale=1 / 64)]
        ins = [oracle.build_input_tables(j) for j in jobs]
        out = c.compact_batch([(i, j.options()) for i, j in zip(ins, jobs)], device_inputs=False)
        for k, (j, i, r) in enumerate(zip(jobs, ins, out)):
            ref = oracle.compact(i, j.options())
            assert r.status == 0, (k, r.name)
            assert_same_files(r.files, ref.files, f"hostsort batch job {k}")
    finally:
        c.set_host_sort(False)


def test_in_place_reads_of_host_and_device_outputs():
    """A function applied to each output table before the library frees it
    sees the same bytes as the copied-out tables: numpy views of host
    outputs (several jobs in one pass: one pinned range each), torch views of
    device outputs."""
    import numpy as np
    import torch
    c = ctx()
    jobs = [tiny_job(40 + s, bottommost=s % 2) for s in range(3)] + [plain_small()]
    ins = [oracle.build_input_tables(j) for j in jobs]
    for k, (j, i) in enumerate(zip(jobs, ins)):
        ref = c.compact(i, j.options())
        view = c.compact(i, j.options(), materialize=lambda a: (type(a), a.tobytes()))
        assert all(t is np.ndarray for t, _ in view.files), k
        assert [b for _, b in view.files] == ref.files, f"host view job {k}"
        dev = [torch.frombuffer(bytearray(b), dtype=torch.uint8).to("cuda") for b in i]
        dview = c.compact_dev(dev, j.options(), materialize=lambda t: t.cpu().numpy().tobytes())
        assert dview.files == ref.files, f"device view job {k}"
    out = c.compact_batch([(i, j.options()) for i, j in zip(ins, jobs)], device_inputs=False,
                          materialize=lambda a: a.tobytes())
    for k, (j, i, r) in enumerate(zip(jobs, ins, out)):
        assert r.files == oracle.compact(i, j.options()).files, f"batched host view job {k}"


def test_pooled_output_buffers_are_reused_and_trimmed():
    """Device outputs of freed results go back to the pool: the next call's
    outputs are the same bytes, and trimming the pool frees them."""
    import torch
    from paper_2004_03054_amd import pool_trim
    c = ctx()
    j = plain_small()
    i = oracle.build_input_tables(j)
    ref = oracle.compact(i, j.options())
    dev = [torch.frombuffer(bytearray(b), dtype=torch.uint8).to("cuda") for b in i]
    for _ in range(3):
        r = c.compact_dev(dev, j.options())
        assert [t.cpu().numpy().tobytes() for t in r.files] == ref.files
    freed = pool_trim(0)
    say(f"[gpu] pool trim freed {freed} bytes")
    assert freed > 0 and pool_trim(0) == 0
    r = c.compact_dev(dev, j.options())
    assert [t.cpu().numpy().tobytes() for t in r.files] == ref.files


def test_contexts_on_threads_share_the_pools():
    """Two contexts used from two host threads at once: staged uploads of
    host inputs (each context's pinned slots and copy threads), results in
    the shared pinned pool and output buffers back in the shared device pool
    give every call the oracle's bytes."""
    import threading
    from paper_2004_03054_amd import Context
    jobs = [plain_large(scale=1 / 16), plain_variable(scale=1 / 16)]  # inputs of 4 MiB or more: the staged path
    ins = [oracle.build_input_tables(j) for j in jobs]
    refs = [oracle.compact(i, j.options()) for i, j in zip(ins, jobs)]
    errors = []

    def work(k):
        try:
            c = Context(0)
            try:
                for rep in range(3):
                    r = c.compact(ins[k], jobs[k].options())
                    assert r.status == 0, (k, rep, r.name)
                    assert_same_files(r.files, refs[k].files, f"thread {k} call {rep}")
            finally:
                c.close()
        except BaseException as e:  # noqa: BLE001 - reported by the main thread
            errors.append(e)

    say("[gpu] two contexts on two threads, 3 calls each")
    th = [threading.Thread(target=work, args=(k,)) for k in range(2)]
    for t in th:
        t.start()
    for t in th:
        t.join(timeout=100)
    assert not any(t.is_alive() for t in th), "a thread did not finish"
    assert not errors, errors[0]


def test_library_before_torch_in_a_fresh_process():
    """A program that creates a context before it touches torch can still use
    torch's device memory afterwards (the binding loads torch's HIP runtime
    first), and compacts device inputs correctly."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = (
        "import sys; sys.path.insert(0, %r); sys.path.insert(0, %r)\n"
        "from paper_2004_03054_amd import Context\n"
        "c = Context(0)\n"
        "import torch, oracle\n"
        "from workload import plain_small\n"
        "j = plain_small(); ins = oracle.build_input_tables(j)\n"
        "dev = [torch.frombuffer(bytearray(b), dtype=torch.uint8).to('cuda') for b in ins]\n"
        "r = c.compact_dev(dev, j.options())\n"
        "ok = [t.cpu().numpy().tobytes() for t in r.files] == oracle.compact(ins, j.options()).files\n"
        "print('same' if ok else 'differ', flush=True)\n"
    ) % (root, os.path.join(root, "tests"))
    say("[gpu] fresh process: context before torch")
    p = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=110)
    assert p.returncode == 0, p.stderr[-2000:]
    assert p.stdout.strip().endswith("same"), p.stdout
