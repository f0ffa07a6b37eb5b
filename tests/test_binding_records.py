"""The batch job records the binding fills with numpy hold what one buffer
list and one options() record per job hold: input pointers and sizes, the
option fields and the snapshot lists (host and torch inputs, empty inputs,
jobs without inputs)."""
import ctypes as C

import numpy as np
import torch

from paper_2004_03054_amd import binding as B


def _jobs(rng, torch_inputs):
    jobs = []
    for j in range(int(rng.integers(1, 12))):
        inp = []
        for _ in range(int(rng.integers(0, 5))):
            n = int(rng.integers(0, 3)) * int(rng.integers(1, 50))
            a = rng.integers(0, 256, n, dtype=np.uint8)
            inp.append(torch.from_numpy(a.copy()) if torch_inputs else (bytes(a) if j % 2 else a))
        o = dict(block_size=int(rng.integers(1, 1 << 20)), restart_interval=int(rng.integers(1, 64)),
                 bloom_bits_per_key=int(rng.integers(0, 20)), bottommost=int(rng.integers(0, 2)),
                 target_file_size=int(rng.integers(1, 1 << 40)))
        if rng.integers(0, 2):
            o["compression"] = 1
        if rng.integers(0, 3) == 0:
            o["snapshots"] = sorted(int(x) for x in rng.integers(0, 1 << 50, int(rng.integers(0, 4))))
        jobs.append((inp, o))
    return jobs


def _check(jobs, cjobs, torch_inputs):
    for j, (inp, o) in enumerate(jobs):
        r = cjobs[j]
        assert r.n_inputs == len(inp)
        bufs = C.cast(r.inputs, C.POINTER(B.LudaBuf))
        for i, t in enumerate(inp):
            n = t.numel() if torch_inputs else len(t)
            assert bufs[i].size == n
            if n == 0:
                assert not bufs[i].data
            else:
                got = C.string_at(bufs[i].data, n)
                want = t.numpy().tobytes() if torch_inputs else bytes(t)
                assert got == want
                if torch_inputs:
                    assert bufs[i].data == t.data_ptr()
        ref = B.options(o)
        for name, _ in B.LudaOptions._fields_:
            if name != "snapshots":
                assert getattr(r.options, name) == getattr(ref, name), (j, name)
        snaps = [int(x) for x in o.get("snapshots", ())]
        assert r.options.n_snapshots == len(snaps)
        if snaps:
            assert [r.options.snapshots[k] for k in range(len(snaps))] == snaps
        else:
            assert not r.options.snapshots


def test_records_match_the_per_job_path():
    rng = np.random.default_rng(5)
    for case in range(40):
        torch_inputs = bool(case % 2)
        jobs = _jobs(rng, torch_inputs)
        cjobs, keep = B.batch_records(jobs, device_inputs=torch_inputs)
        _check(jobs, cjobs, torch_inputs)


def test_empty_batch():
    cjobs, keep = B.batch_records([], device_inputs=True)
    assert C.sizeof(cjobs) == C.sizeof(B.LudaJob)


def _fake_results(rng, J):
    res = (B.LudaResult * max(1, J))()
    keep = []
    for j in range(J):
        r = res[j]
        r.status = int(rng.choice([0, 0, 0, 3]))
        r.error.status, r.error.input, r.error.where, r.error.phase = (int(x) for x in rng.integers(0, 9, 4))
        r.error.block, r.error.offset = (int(x) for x in rng.integers(0, 1 << 40, 2))
        for k in ("entries_in", "entries_out", "dropped_shadowed", "dropped_tombstones", "bytes_in", "bytes_out"):
            setattr(r, k, int(rng.integers(0, 1 << 50)))
        r.ms_total = float(rng.random())
        nf = int(rng.integers(0, 5))
        if nf:
            fs = (B.LudaFile * nf)()
            for f in fs:
                f.offset, f.size, f.num_entries = (int(x) for x in rng.integers(0, 1 << 40, 3))
                f.smallest_off = f.offset + int(rng.integers(0, 1000))
                f.largest_off = f.offset + int(rng.integers(0, 1000))
                f.smallest_len, f.largest_len = (int(x) for x in rng.integers(0, 100, 2))
            keep.append(fs)
            r.files = C.cast(fs, C.POINTER(B.LudaFile))
            r.num_files = nf
    return res, keep


def test_batch_results_match_the_per_job_path(monkeypatch):
    """take_records gives the Result that _take gives without output bytes,
    and hands every record back once."""
    import types
    monkeypatch.setattr(B, "lib", lambda: types.SimpleNamespace(luda_result_free=lambda *a: None))
    rng = np.random.default_rng(9)
    for J in (0, 1, 7, 40):
        res, keep = _fake_results(rng, J)
        freed = []
        got = B.take_records(res, J, lambda r: freed.append(C.addressof(r)))
        want = [B._take(None, res[j], device=True, materialize=False) for j in range(J)]
        assert got == want
        assert freed == [C.addressof(res[j]) for j in range(J)]
