"""Benchmark: compaction input GB/s of the batched form against the plain
per-job calls, and p99 job latency of the served form, on one MI355X.

Default run (the headline):

* Batch workload: 256 independent jobs, each 1 upper + U{1..12} lower tables
  of U{2..64} MiB (about 59 GiB in all), 16-byte keys uniform over the job's
  range, values U{100..1024} B, 5% deletions, 4 KiB blocks, restart interval
  16, 10 bits/key Bloom filters, 64 MiB output tables, bottom level on even
  jobs.  The tables are written on the GPU by the library's own table writer
  from seeded synthetic entries and stay resident in HBM.  One step is one
  batched pass over all 256 jobs (decode with checksums, merge and drop,
  re-encode with index, filter and checksums), outputs left in HBM.  `value`
  is input bytes / wall time of the timed passes; the same jobs run as one
  plain call per job give `plain_loop_gbps`.
* Served record: Poisson arrivals at 200 jobs/s of jobs drawn from the same
  pool, through the request loop and through plain per-job launches, with
  outputs copied to host memory: p50 / p99 latency and sustained GB/s.
* Plain record: the large single compaction (1 upper + 10 lower tables of
  64 MiB, Zipf keys, 1 KiB values), kernel-only and end to end.
* cpu_baseline: the plain oracle on the host cores (one batch job per
  thread), bit-exact against the GPU on the same jobs.

Other modes (--mode plain|batch|serve|coopsort|copy) run one part alone.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def device_tables(ctx, job):
    """Write each run of the job as one input table on the GPU."""
    import torch
    tables = []
    for r in job.runs:
        t = lambda a: torch.from_numpy(a).to("cuda")  # noqa: E731
        keys = t(r.keys if r.keys.size else r.keys.reshape(0))
        res = ctx.build_tables_dev(t(r.keys), t(r.koff.astype("int64")), t(r.tags.view("int64")),
                                   t(r.vals), t(r.voff.astype("int64")), job.table_options())
        if res.status != 0 or len(res.files) != 1:
            raise RuntimeError(f"device table writer failed: {res.name} {ctx.last_error()}")
        tables.append(res.files[0])
        del keys
    torch.cuda.synchronize()
    return tables


def fingerprint(t) -> int:
    """A 64-bit fingerprint of device bytes (for comparing outputs without
    copying them to the host)."""
    import torch
    n = t.numel()
    pad = (-n) % 8
    if pad:
        t = torch.cat([t, torch.zeros(pad, dtype=torch.uint8, device=t.device)])
    w = t.view(torch.int64)
    idx = torch.arange(w.numel(), dtype=torch.int64, device=t.device)
    mult = idx * 0x5851F42D4C957F2D + 0x14057B7EF767814F  # wraps mod 2^64
    return int(((w ^ (w >> 29)) * (mult | 1)).sum().item()) ^ n


# rocprofv3 byte counters of a kernel are valid only for the sources they
# were taken on: profiles/ records them with a hash of those sources
TRAFFIC_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles", "traffic_plain_large_11x64MiB.md")
TRAFFIC_SOURCES = ["k_encode.hip", "dev_common.h", "kernels.h", "luda_internal.h", "crc_multi.h"]


BATCH_TRAFFIC_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles", "traffic_batch_256jobs.md")


def measured_traffic(kernel: str, path: str = TRAFFIC_FILE):
    """HBM bytes per launch of `kernel` from a committed counter summary,
    or None when it is missing or the kernel's sources changed since."""
    import hashlib
    import re
    try:
        text = open(path).read()
    except OSError:
        return None
    m = re.search(r"^traffic %s bytes_per_launch=(\d+) sources_sha256=([0-9a-f]+)$" % re.escape(kernel), text, re.M)
    if not m:
        return None
    h = hashlib.sha256()
    csrc = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2004_03054_amd", "csrc")
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return float(m.group(1)) if h.hexdigest() == m.group(2) else None


def host_fingerprint(b: bytes, full: bool = True) -> tuple:
    """A fingerprint of host bytes for comparing outputs: word sums over all
    8-byte words (full) or over every 512th word.  Vectorised, unlike a
    cryptographic hash, so that it keeps up with the GPU."""
    import numpy as np
    n = len(b) // 8
    v = np.frombuffer(b, dtype=np.uint64, count=n)
    if not full:
        v = v[::512]
    return len(b), int(v.sum(dtype=np.uint64)), int(v[1::2].sum(dtype=np.uint64)), bytes(b[8 * n:])


def host_info() -> dict:
    """The host the oracle ran on: logical CPUs and CPU model."""
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "cpu_model": model}


def kernel_times(ctx):
    """Device time of each timed kernel in the last call (launches of the same
    kernel, e.g. merge rounds, summed).  The encoder is two kernels (the
    pipelined blocks, then the large ones): "k_encode" is their sum, and
    "k_encode_big" is also given alone."""
    out = {}
    for k, v in ctx.stage_times():
        if k.startswith("kernel:"):
            name = k.split(":", 1)[1]
            out[name] = out.get(name, 0.0) + v
            if name == "k_encode_big":
                out["k_encode"] = out.get("k_encode", 0.0) + v
    return out


def parse_args(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--scale", type=float, default=1.0, help="table size scale (1.0 = the stated sizes)")
    ap.add_argument("--workload", choices=["small", "large", "variable"], default="large",
                    help="plain mode: small (3 x 10k entries), large (11 x 64 MiB), variable-size keys and values "
                         "(7 x 32 MiB)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--e2e-steps", type=int, default=3)
    ap.add_argument("--copy-mib", type=int, default=1024, help="copy mode: bytes copied per launch (MiB)")
    ap.add_argument("--mode", choices=["headline", "plain", "batch", "serve", "copy", "coopsort", "batchpass"],
                    default="headline",
                    help="headline (default): batched vs plain on the 256-job batch workload, with a served "
                         "record at 200 jobs/s and the plain large compaction as sub-records; plain: one large "
                         "compaction; batch: the batched pass vs a loop of plain calls; serve: Poisson arrivals "
                         "through the request loop vs plain per-job launches; batchpass: batched passes only, for "
                         "profiling; copy: a device copy, for scaling byte counters")
    ap.add_argument("--rate", type=str, default="50",
                    help="serve mode: arrivals per second (a comma-separated list runs each on one job pool)")
    ap.add_argument("--workers", type=int, default=2, help="serve mode: the served form's workers")
    ap.add_argument("--duration", type=float, default=10.0, help="serve mode: seconds of arrivals")
    ap.add_argument("--budget-gib", type=float, default=64.0, help="serve mode: HBM budget")
    ap.add_argument("--max-batch", type=int, default=None,
                    help="serve mode: most jobs in one pass of the request loop (0: no limit); default 1 with "
                         "outputs copied to host memory (the host link bounds the rate, and a larger pass only "
                         "delays its first copy), 16 with outputs kept in HBM")
    ap.add_argument("--keep-s", type=float, default=3.0,
                    help="serve --resident: outputs of requests that arrived up to this many seconds earlier "
                         "stay in HBM as inputs of later requests")
    ap.add_argument("--resident", action="store_true",
                    help="serve mode: outputs stay in HBM and half the requests read an earlier request's outputs")
    ap.add_argument("--jobs", type=int, default=256, help="batch mode: number of jobs")
    ap.add_argument("--oracle-jobs", type=int, default=0,
                    help="batch mode: jobs checked against the oracle and timed on the host cores "
                         "(default: one per oracle thread)")
    ap.add_argument("--oracle-threads", type=int, default=0,
                    help="batch mode: host threads running oracle jobs at once (default: the host's cores, at most 16)")
    ap.add_argument("--serve-rate", type=float, default=200.0, help="headline: arrival rate of the served record")
    ap.add_argument("--serve-duration", type=float, default=20.0, help="headline: seconds of arrivals")
    return ap.parse_args(argv)


def main():
    args = parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (jobs are independent: "
              "several GPUs would each run their own jobs with no exchange)", file=sys.stderr)
        sys.exit(2)
    if args.mode == "headline":
        return headline_main(args)
    if args.mode == "batch":
        return batch_main(args)
    if args.mode == "serve":
        return serve_main(args)
    if args.mode == "copy":
        return copy_main(args)
    if args.mode == "coopsort":
        return coopsort_main(args)
    if args.mode == "batchpass":
        return batchpass_main(args)
    out = plain_record(args, args.workload, args.scale, args.steps, args.warmup, not args.no_cpu_baseline,
                       args.e2e_steps)
    print(json.dumps(out), flush=True)


def plain_alg_bytes(counters: dict) -> dict:
    """Algorithmic bytes per launch of the timed kernels:
    k_crc_data reads every input data block once (contents + trailer);
    k_encode reads every surviving value once and writes every output data
    block once (both approximated by the output data-block bytes);
    k_walk_emit writes one 36-byte entry record per input entry;
    k_keys reads 16 bytes of record per entry, writes its key slot
    (8 * kw8 bytes) and 28 bytes of sort keys."""
    n_in = counters.get("entries_in", 0.0)
    kw8 = counters.get("kw8", 2.0)
    return {
        "k_crc_data": counters.get("data_bytes_in", 0.0),
        "k_encode": 2.0 * counters.get("data_bytes_out", 0.0),
        "k_walk_emit": 36.0 * n_in,
        "k_keys": n_in * (16.0 + 8.0 * kw8 + 28.0),
    }


def roofline_of(kavg: dict, alg: dict, traffic=None) -> tuple:
    """(roofline of the dominant kernel by time, per-kernel rates)."""
    dom = max(alg, key=lambda k: kavg.get(k, 0.0))
    achieved = alg[dom] / (kavg[dom] * 1e-3) / 1e9 if kavg.get(dom) else 0.0
    roof = {"kernel": dom, "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic(dom) if traffic else None,
            "alg_bytes_per_launch": alg[dom], "avg_ms": round(kavg.get(dom, 0.0), 4)}
    other = {k: {"avg_ms": round(kavg.get(k, 0.0), 4),
                 "gbps": round(alg[k] / (kavg[k] * 1e-3) / 1e9, 1) if kavg.get(k) else None}
             for k in alg}
    return roof, other


def plain_record(args, workload, scale, steps, warmup, cpu_baseline=True, e2e_steps=3):
    """One plain compaction of a plain workload, inputs resident in HBM,
    timed over `steps` calls; end to end and the oracle beside it."""
    import numpy as np
    import torch
    from paper_2004_03054_amd import Context
    from workload import plain_small, plain_large, plain_variable

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    t0 = time.time()
    job = {"small": lambda: plain_small(), "large": lambda: plain_large(scale=scale),
           "variable": lambda: plain_variable(scale=scale)}[workload]()
    log(f"[bench] generated {job.name}: {sum(r.n for r in job.runs)} entries in {time.time() - t0:.1f}s")
    ctx = Context(0)
    tables = device_tables(ctx, job)
    in_bytes = sum(int(t.numel()) for t in tables)
    log(f"[bench] {len(tables)} input tables on the device, {in_bytes / 2**20:.1f} MiB")
    opts = job.options()

    # warmup (also checks the result is well formed)
    res = None
    for _ in range(warmup):
        res = ctx.compact_dev(tables, opts, materialize=False)
        assert res.status == 0, (res.name, ctx.last_error())
    # timed steps: kernel-only (inputs resident in HBM, outputs left in HBM)
    ktimes = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    step_s = []
    for _ in range(steps):
        ts = time.perf_counter()
        res = ctx.compact_dev(tables, opts, materialize=False)  # returns after its stream is done
        step_s.append(time.perf_counter() - ts)
        ktimes.append(kernel_times(ctx))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t_start
    assert res.status == 0, (res.name, ctx.last_error())
    counters = ctx.counters()
    ms_step = dt * 1e3 / steps
    value = in_bytes * steps / dt / 1e9
    log(f"[bench] {job.name}: {steps} steps: {ms_step:.3f} ms/step, {value:.1f} GB/s input")

    names = sorted(set(k for kt in ktimes for k in kt))
    kavg = {n: float(np.mean([kt.get(n, 0.0) for kt in ktimes])) for n in names}
    # the committed counters were taken on the large workload only
    traffic = measured_traffic if (workload == "large" and scale == 1.0) else None
    roofline, other = roofline_of(kavg, plain_alg_bytes(counters), traffic)
    roofline["path"] = path_roofline(in_bytes, res.bytes_out, ms_step)

    # end to end: host tables in, host tables out (PCIe both ways): the
    # library's C-ABI from host input buffers to its host result buffers
    # (the binding's copy of them into Python objects is left out)
    host_tables = [t.cpu().numpy().tobytes() for t in tables]
    e2e = None
    if e2e_steps > 0:
        r = ctx.compact(host_tables, opts, materialize=False)
        assert r.status == 0
        t1 = time.perf_counter()
        for _ in range(e2e_steps):
            r = ctx.compact(host_tables, opts, materialize=False)
            assert r.status == 0
        e2e_dt = time.perf_counter() - t1
        e2e = round(in_bytes * e2e_steps / e2e_dt / 1e9, 2)
        log(f"[bench] end to end: {e2e} GB/s")
    gpu_files = ctx.compact(host_tables, opts).files

    cpu = None
    if cpu_baseline:
        # the oracle (plain sequential C, one thread) on the same workload:
        # its own input tables, timed around the compaction only
        import oracle
        ref_inputs = oracle.build_input_tables(job)
        same_inputs = ref_inputs == host_tables
        t2 = time.perf_counter()
        ref = oracle.compact(ref_inputs, opts)
        cdt = time.perf_counter() - t2
        digest = lambda fs: hashlib.sha256(b"".join(fs)).hexdigest()  # noqa: E731
        cpu = {"value": round(in_bytes / cdt / 1e9, 4), "unit": "GB/s", "cores": 1, "kind": "oracle",
               "sample": f"one full compaction of the same workload ({in_bytes / 2**20:.0f} MiB input), "
                         f"{cdt:.1f} s",
               "bit_exact": bool(ref.status == 0 and ref.files == gpu_files),
               "inputs_identical": bool(same_inputs), "host": host_info(),
               "sha256_gpu": digest(gpu_files)[:16], "sha256_oracle": digest(ref.files)[:16]}
        log(f"[bench] oracle: {cdt:.1f}s, bit-exact {cpu['bit_exact']}")
    ctx.close()
    return {
        "metric": "compaction input GB/s",
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": job.name, "inputs": len(tables), "input_bytes": in_bytes,
                   "entries_in": res.entries_in, "entries_out": res.entries_out,
                   "files_out": len(res.file_sizes), "block_size": opts["block_size"],
                   "restart_interval": opts["restart_interval"], "bloom_bits_per_key": opts["bloom_bits_per_key"],
                   "bottommost": opts["bottommost"], "target_file_size": opts["target_file_size"],
                   "inputs_resident": "hbm", "outputs": "hbm"},
        "step_ms": {"median": round(float(np.median(step_s)) * 1e3, 4), "min": round(min(step_s) * 1e3, 4),
                    "p90": round(float(np.percentile(step_s, 90)) * 1e3, 4)},
        "end_to_end_gbps": e2e,
        "kernel_ms": {k: round(v, 4) for k, v in kavg.items()},
        "kernels": other,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }


def path_roofline(in_bytes: float, out_bytes: float, ms: float) -> dict:
    """The whole call against the HBM peak: its algorithmic bytes (every input
    byte read once, every output byte written once) over the call's time."""
    gbps = (in_bytes + out_bytes) / (ms * 1e-3) / 1e9 if ms else 0.0
    return {"alg_bytes": in_bytes + out_bytes, "achieved": round(gbps, 1), "frac": round(gbps / HBM_PEAK_GBS, 4)}


def build_batch_pool(ctx, n_jobs, scale):
    """The batch workload's jobs written as device tables (resident in HBM)."""
    from workload import batch_job
    jobs, tables, in_bytes = [], [], 0
    t0 = time.time()
    for j in range(n_jobs):
        job = batch_job(j, scale=scale)
        tabs = device_tables(ctx, job)
        tables.append(tabs)
        jobs.append((job.name, job.options()))
        in_bytes += sum(int(t.numel()) for t in tabs)
        del job
        if (j + 1) % 32 == 0:
            log(f"[bench] {j + 1} jobs on the device, {in_bytes / 2**30:.2f} GiB, {time.time() - t0:.0f}s")
    log(f"[bench] {n_jobs} jobs, {in_bytes / 2**30:.2f} GiB of input tables resident ({time.time() - t0:.0f}s)")
    return jobs, tables, in_bytes


def batch_alg_bytes(counters: dict) -> dict:
    return plain_alg_bytes(counters)


def oracle_on_batch_jobs(ctx, tables, scale, n_oracle, threads):
    """The oracle on the host cores: independent jobs of the batch on
    `threads` threads at once (the oracle is C called through ctypes, which
    runs without the interpreter lock), aggregate input GB/s; every job is
    also checked byte for byte against the GPU."""
    from concurrent.futures import ThreadPoolExecutor
    import oracle
    from workload import batch_job as mk

    def prep(j):
        job = mk(j, scale=scale)
        return job.options(), oracle.build_input_tables(job)

    with ThreadPoolExecutor(max_workers=threads) as ex:
        prepared = list(ex.map(prep, range(n_oracle)))

    def run_one(k):
        return oracle.compact(prepared[k][1], prepared[k][0])

    t2 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        refs = list(ex.map(run_one, range(n_oracle)))
    tot_t = time.perf_counter() - t2
    tot_b = sum(sum(len(x) for x in p[1]) for p in prepared)
    exact = True
    for j in range(n_oracle):
        host = [t.cpu().numpy().tobytes() for t in tables[j]]
        r = ctx.compact(host, prepared[j][0])
        exact = exact and prepared[j][1] == host and refs[j].status == 0 and refs[j].files == r.files
    cores = min(threads, n_oracle)
    cpu = {"value": round(tot_b / tot_t / 1e9, 4), "unit": "GB/s", "cores": cores, "kind": "oracle",
           "sample": f"jobs 0..{n_oracle - 1} of the batch ({tot_b / 2**20:.0f} MiB) on {cores} threads at once, "
                     f"{tot_t:.1f} s wall",
           "bit_exact": bool(exact), "inputs_identical": bool(exact), "host": host_info()}
    log(f"[bench] oracle: {n_oracle} jobs on {cores} threads in {tot_t:.1f}s, bit-exact {exact}")
    return cpu


def batch_record(args, ctx, jobs, tables, in_bytes, steps, warmup, scale):
    """The batched pass against one plain call per job, on the same resident
    jobs; outputs of the two compared job by job (device fingerprints)."""
    import numpy as np
    import torch
    batch = [(tables[j], jobs[j][1]) for j in range(len(jobs))]
    # launch parameters from the autotuner, on a sample of the jobs
    tuned, tuned_ms = ctx.autotune(batch[:min(8, len(jobs))], device_inputs=True, rounds=1)
    log(f"[bench] autotuned launch parameters {tuned} ({tuned_ms:.1f} ms on the sample)")
    # verification pass (outside timing): batched outputs == per-job outputs
    res_b = ctx.compact_batch(batch, device_inputs=True, materialize=fingerprint)
    fp_b = [r.files for r in res_b]
    status_b = [r.status for r in res_b]
    del res_b
    fp_p = []
    for j in range(len(jobs)):
        r = ctx.compact_dev(tables[j], jobs[j][1], materialize=fingerprint)
        fp_p.append(r.files)
        assert r.status == 0 and status_b[j] == 0, (j, r.name, ctx.last_error())
    same = fp_p == fp_b
    log(f"[bench] batched outputs identical to per-job outputs: {same}")
    torch.cuda.synchronize()
    # warmup, then timed: plain loop, then batched
    for _ in range(max(0, warmup)):
        out = ctx.compact_batch(batch, device_inputs=True, materialize=False)
    plain_steps = max(1, min(steps, 5))
    torch.cuda.synchronize()
    tp = time.perf_counter()
    for _ in range(plain_steps):
        for j in range(len(jobs)):
            ctx.compact_dev(tables[j], jobs[j][1], materialize=False)
    torch.cuda.synchronize()
    plain_s = (time.perf_counter() - tp) / plain_steps
    ktimes, counters, out_bytes = [], None, 0
    torch.cuda.synchronize()
    tb = time.perf_counter()
    for _ in range(steps):
        out = ctx.compact_batch(batch, device_inputs=True, materialize=False)
        ktimes.append(kernel_times(ctx))
    torch.cuda.synchronize()
    batch_s = (time.perf_counter() - tb) / steps
    assert all(r.status == 0 for r in out)
    counters = ctx.counters()
    out_bytes = sum(r.bytes_out for r in out)
    value = in_bytes / batch_s / 1e9
    plain = in_bytes / plain_s / 1e9
    log(f"[bench] batched {batch_s * 1e3:.1f} ms ({value:.1f} GB/s), plain loop {plain_s * 1e3:.1f} ms "
        f"({plain:.1f} GB/s)")
    names = sorted(set(k for kt in ktimes for k in kt))
    kavg = {n: float(np.mean([kt.get(n, 0.0) for kt in ktimes])) for n in names}
    traffic = (lambda k: measured_traffic(k, BATCH_TRAFFIC_FILE)) if (scale == 1.0 and len(jobs) == 256) else None
    roofline, other = roofline_of(kavg, batch_alg_bytes(counters), traffic)
    roofline["path"] = path_roofline(in_bytes, out_bytes, batch_s * 1e3)
    return dict(value=value, batch_s=batch_s, plain=plain, plain_s=plain_s, plain_steps=plain_steps, same=same,
                tuned=tuned, kavg=kavg, kernels=other, roofline=roofline, out_bytes=out_bytes,
                counters=counters)


def headline_main(args):
    """The metric as stated: batched vs plain on the batch workload, the
    served form's p50 / p99 at 200 jobs/s on the same job pool, and the plain
    large compaction; one JSON line."""
    import numpy as np  # noqa: F401
    import torch
    from paper_2004_03054_amd import Context

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    t_all = time.time()
    ctx = Context(0)
    jobs, tables, in_bytes = build_batch_pool(ctx, args.jobs, args.scale)
    b = batch_record(args, ctx, jobs, tables, in_bytes, args.steps, args.warmup, args.scale)
    cpu = None
    if not args.no_cpu_baseline:
        threads = args.oracle_threads or min(16, os.cpu_count() or 1)
        cpu = oracle_on_batch_jobs(ctx, tables, args.scale, min(args.oracle_jobs or threads, len(jobs)), threads)
    # served form on the same pool: Poisson arrivals, host outputs
    tbytes = [sum(int(t.numel()) for t in tabs) for tabs in tables]
    served = serve_record(args, tables, [o for _, o in jobs], tbytes, args.serve_rate, args.serve_duration,
                          resident=False, max_batch=1, workers=2, budget_gib=64.0, keep_s=args.keep_s)
    ctx.close()
    del tables
    torch.cuda.empty_cache()
    plain = plain_record(args, "large", 1.0, args.steps, args.warmup, not args.no_cpu_baseline, args.e2e_steps)
    out = {
        "metric": "compaction input GB/s (batched vs plain, bit-exact SSTs); p99 job latency",
        "value": round(b["value"], 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(b["batch_s"] * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": f"batch-{args.jobs}-jobs" + ("" if args.scale == 1.0 else f"-scale{args.scale:g}"),
                   "jobs": args.jobs, "input_bytes": in_bytes, "output_bytes": b["out_bytes"],
                   "entries_in": b["counters"].get("entries_in"), "survivors": b["counters"].get("survivors"),
                   "block_size": 4096, "restart_interval": 16, "bloom_bits_per_key": 10,
                   "target_file_size": 64 << 20, "inputs_resident": "hbm", "outputs": "hbm"},
        "plain_loop_gbps": round(b["plain"], 2),
        "plain_loop_ms": round(b["plain_s"] * 1e3, 2),
        "batched_over_plain": round(b["plain_s"] / b["batch_s"], 3),
        "outputs_identical": bool(b["same"]),
        "launch_params": b["tuned"],
        "kernel_ms": {k: round(v, 4) for k, v in b["kavg"].items()},
        "kernels": b["kernels"],
        "roofline": b["roofline"],
        "cpu_baseline": cpu,
        "served": served,
        "plain_large": plain,
        "bench_wall_s": round(time.time() - t_all, 1),
    }
    print(json.dumps(out), flush=True)


def batch_main(args):
    """Many independent uneven jobs: one batched pass over every stage vs one
    plain call per job, on the same device-resident inputs."""
    import torch
    from paper_2004_03054_amd import Context

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    ctx = Context(0)
    jobs, tables, in_bytes = build_batch_pool(ctx, args.jobs, args.scale)
    b = batch_record(args, ctx, jobs, tables, in_bytes, max(1, args.steps), 1, args.scale)
    cpu = None
    threads = args.oracle_threads or min(16, os.cpu_count() or 1)
    n_oracle = min(args.oracle_jobs or threads, len(tables))
    if n_oracle > 0 and not args.no_cpu_baseline:
        cpu = oracle_on_batch_jobs(ctx, tables, args.scale, n_oracle, threads)
    out = {
        "metric": "compaction input GB/s (batched)",
        "value": round(b["value"], 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": max(1, args.steps),
        "warmup": 1,
        "ms_per_step": round(b["batch_s"] * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": f"batch-{args.jobs}-jobs" + ("" if args.scale == 1.0 else f"-scale{args.scale:g}"),
                   "jobs": args.jobs, "input_bytes": in_bytes, "inputs_resident": "hbm", "outputs": "hbm"},
        "plain_loop_gbps": round(b["plain"], 2),
        "batched_over_plain": round(b["plain_s"] / b["batch_s"], 3),
        "outputs_identical": bool(b["same"]),
        "launch_params": b["tuned"],
        "kernel_ms": {k: round(v, 4) for k, v in b["kavg"].items()},
        "roofline": b["roofline"],
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    ctx.close()


def coopsort_main(args):
    """The paper's cooperative sort against the device merge, on the plain
    large compaction: the same resident tables compacted with the merge step
    on the device, then with the entries' keys copied to the host, sorted on
    host threads and the order copied back.  Reports both step times and the
    merge stage (HIP events around it), and checks the outputs are the same
    bytes (device fingerprints)."""
    os.environ["LUDA_STAGE_TIMES"] = "1"
    import numpy as np
    import torch
    from paper_2004_03054_amd import Context
    from workload import plain_large

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    job = plain_large(scale=args.scale)
    ctx = Context(0)
    tables = device_tables(ctx, job)
    in_bytes = sum(int(t.numel()) for t in tables)
    opts = job.options()
    out = {}
    prints = {}
    for name, host in (("device_merge", False), ("host_sort", True)):
        ctx.set_host_sort(host)
        for _ in range(args.warmup):
            r = ctx.compact_dev(tables, opts, materialize=False)
            assert r.status == 0, (r.name, ctx.last_error())
        steps, merge = [], []
        for _ in range(args.steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = ctx.compact_dev(tables, opts, materialize=False)
            torch.cuda.synchronize()
            steps.append((time.perf_counter() - t0) * 1e3)
            st = dict(ctx.stage_times())
            merge.append(st.get("merge", float("nan")))
        r = ctx.compact_dev(tables, opts, materialize=fingerprint)
        prints[name] = [f for f in r.files]
        out[name] = {"ms_per_step": round(float(np.median(steps)), 3),
                     "merge_stage_ms": round(float(np.median(merge)), 3),
                     "gbps": round(in_bytes / (np.median(steps) * 1e-3) / 1e9, 1)}
        log(f"[bench] {name}: {out[name]}")
    ctx.set_host_sort(False)
    print(json.dumps({"mode": "coopsort", "workload": job.name, "input_bytes": in_bytes,
                      "entries_in": int(sum(r.n for r in job.runs)), "host_threads": min(16, os.cpu_count() or 1),
                      "device_merge": out["device_merge"], "host_sort": out["host_sort"],
                      "outputs_identical": prints["device_merge"] == prints["host_sort"]}), flush=True)


def batchpass_main(args):
    """The batched pass alone (for profiling): build the batch workload's
    tables on the device, then `--steps` batched passes; one JSON line of
    their times.  No plain loop, no verification, no oracle."""
    import torch
    from paper_2004_03054_amd import Context

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    ctx = Context(0)
    jobs, tables, in_bytes = build_batch_pool(ctx, args.jobs, args.scale)
    batch = [(tables[j], jobs[j][1]) for j in range(len(jobs))]
    ms = []
    for _ in range(max(1, args.steps)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = ctx.compact_batch(batch, device_inputs=True, materialize=False)
        torch.cuda.synchronize()
        ms.append((time.perf_counter() - t0) * 1e3)
        assert all(r.status == 0 for r in out)
        del out
    print(json.dumps({"mode": "batchpass", "jobs": len(jobs), "input_bytes": in_bytes,
                      "ms_per_pass": [round(x, 3) for x in ms]}), flush=True)
    ctx.close()


def copy_main(args):
    """A plain device copy of known size: the reference for scaling the
    hardware byte counters (FETCH_SIZE / WRITE_SIZE) of the other kernels."""
    import torch
    n = args.copy_mib << 20
    a = torch.randint(0, 255, (n,), dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(max(1, args.steps)):
        b.copy_(a)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / max(1, args.steps)
    print(json.dumps({"mode": "copy", "bytes_read_per_launch": n, "bytes_written_per_launch": n,
                      "launches": max(1, args.steps), "ms_per_launch": round(dt * 1e3, 4),
                      "gbps_read_plus_write": round(2 * n / dt / 1e9, 1)}), flush=True)


def run_trace(srv, arrivals, picks, tables, opts, tbytes, sub=None, keep_s=3.0):
    """Submit each request at its arrival time; collect in order.  Returns
    per-request (latency ms from the arrival time, input bytes, output
    digest) and the span.  With
    sub, request k whose sub[k] is an earlier request k2 takes k2's output
    tables (left in HBM by the server) in place of its first lower input; it
    waits for k2 if k2 is not done yet.  Outputs of requests that arrived more
    than keep_s seconds before the current one are dropped."""
    import threading
    tickets = [None] * len(arrivals)
    ready = threading.Semaphore(0)
    out = [None] * len(arrivals)
    files = [None] * len(arrivals)
    done = [threading.Event() for _ in arrivals]

    failed = []

    def collect():
        try:
            collect_all()
        except BaseException as e:  # noqa: BLE001 - handed to the submitting thread
            failed.append(e)
            for ev in done:
                ev.set()
            for _ in range(len(arrivals)):
                ready.release()

    def collect_all():
        for k in range(len(arrivals)):
            ready.acquire()
            # every 32nd request's outputs are fingerprinted, in place before
            # the library frees them (fingerprinting every result in Python
            # would not keep up with the GPU, and its pauses would delay the
            # submitting thread); the others are compared by file sizes
            sample = k % 32 == 0
            if sub is None:  # host outputs
                r, lat = srv.poll(tickets[k], materialize=host_fingerprint if sample else False)
                assert r.status == 0, (k, r.name)
                dig = repr(r.files) if sample else repr(r.file_sizes)
            else:  # device outputs, kept as inputs of later requests
                r, lat = srv.poll(tickets[k])
                assert r.status == 0, (k, r.name)
                files[k] = r.files
                dig = repr([fingerprint(t) for t in r.files]) if sample else repr(r.file_sizes)
            out[k] = (lat + lag[k], inb[k], dig, time.perf_counter())
            done[k].set()
            if (k + 1) % 250 == 0:
                log(f"[bench] {k + 1} of {len(arrivals)} requests done")

    inb = [0] * len(arrivals)
    lag = [0.0] * len(arrivals)
    th = threading.Thread(target=collect, daemon=True)
    th.start()
    t0 = time.perf_counter()
    for k, (at, j) in enumerate(zip(arrivals, picks)):
        if failed:
            break
        d = at - (time.perf_counter() - t0)
        if d > 0:
            time.sleep(d)
        ins = tables[j]
        if sub is not None and sub[k] is not None:
            done[sub[k]].wait()
            if failed:
                break
            ins = [ins[0]] + list(files[sub[k]]) + list(ins[2:])
        if sub is not None:  # outputs no later request can read
            for q in range(k):
                if arrivals[q] < at - keep_s and done[q].is_set():
                    files[q] = None
        inb[k] = sum(int(t.numel()) for t in ins)
        lag[k] = max(0.0, time.perf_counter() - t0 - at) * 1e3  # submitted late by this thread
        tickets[k] = srv.submit(ins, opts[j])
        ready.release()
    th.join()
    if failed:
        raise RuntimeError("a served request failed") from failed[0]
    span = max(o[3] for o in out) - t0
    return out, span


def serve_record(args, tables, opts, tbytes, rate, duration, resident, max_batch, workers, budget_gib, keep_s):
    """One seeded Poisson trace at `rate` jobs/s through the request loop
    (served) and through plain per-job launches (one worker, one job per
    pass).  Latency = completion (outputs in host memory; in HBM with
    resident) minus arrival, after a start-up interval; every job's outputs
    compared between the two forms."""
    import numpy as np
    from paper_2004_03054_amd import Server
    rng = np.random.default_rng(0x5E5E)
    n = max(1, int(rate * duration))
    arrivals = np.cumsum(rng.exponential(1.0 / rate, n)).tolist()
    picks = rng.integers(0, len(tables), n).tolist()
    budget = int(budget_gib * 2**30)
    sub = None
    if resident:
        # with probability 1/2 a request's first lower input is replaced by the
        # output tables of a request that arrived at least 1 s earlier
        # (from the last keep_s seconds of arrivals, so that older outputs can be freed)
        sub = []
        for k, at in enumerate(arrivals):
            early = [q for q in range(k) if at - keep_s <= arrivals[q] <= at - 1.0]
            sub.append(int(rng.choice(early)) if early and rng.random() < 0.5 else None)
        log(f"[bench] {sum(x is not None for x in sub)} of {n} requests read earlier outputs kept in HBM")
    results = {}
    for name, kw in (("served", dict(max_batch_jobs=max_batch, workers=workers)),
                     ("plain", dict(max_batch_jobs=1, workers=1))):
        srv = Server(0, hbm_budget=budget, host_outputs=not resident, **kw)
        # warm the workers' buffers on the largest job
        big = int(np.argmax(tbytes))
        srv.poll(srv.submit(tables[big], opts[big]))
        out, span = run_trace(srv, arrivals, picks, tables, opts, tbytes, sub, keep_s)
        st = srv.stats()
        mem = srv.memory()
        srv.close()
        lat = np.array([o[0] for o in out])
        warm = np.array(arrivals) >= min(2.0, duration * 0.2)  # drop the start-up interval
        lw = lat[warm] if warm.any() else lat
        results[name] = dict(p50_ms=round(float(np.percentile(lw, 50)), 3),
                             p99_ms=round(float(np.percentile(lw, 99)), 3),
                             gbps=round(sum(o[1] for o in out) / span / 1e9, 3), jobs=n, batches=st["batches"],
                             max_batch=st["max_batch"], peak_admitted_gib=round(st["peak_admitted"] / 2**30, 2),
                             workers_held_gib=round(mem["held_by_workers"] / 2**30, 2),
                             device_used_gib=round(mem["device_used"] / 2**30, 2),
                             digests=[o[2] for o in out])
        log(f"[bench] {name} at {rate:g}/s: p50 {results[name]['p50_ms']} ms, p99 {results[name]['p99_ms']} ms, "
            f"{results[name]['gbps']} GB/s, {st['batches']} passes")
        slow = np.argsort(lat)[-5:][::-1]
        log(f"[bench] {name} slowest (request, arrival s, input MiB, ms): " +
            ", ".join(f"({int(q)}, {arrivals[q]:.2f}, {out[q][1] / 2**20:.0f}, {lat[q]:.1f})" for q in slow))
    same = results["served"].pop("digests") == results["plain"].pop("digests")
    log(f"[bench] every served job's outputs identical to its plain run: {same}")
    return {"rate_per_s": rate, "duration_s": duration, "hbm_budget_gib": budget_gib, "max_batch_jobs": max_batch,
            "workers": workers, "outputs": "hbm" if resident else "host", "resident_inputs": bool(resident),
            **({"keep_s": keep_s} if resident else {}),
            "served": results["served"], "plain_per_job": results["plain"], "outputs_identical": bool(same)}


def serve_main(args):
    """Poisson arrivals of jobs drawn from the batch workload's job mixture,
    through the request loop (admission under an HBM budget, batched passes
    on two workers) and through plain per-job launches (one job at a time),
    on the same trace.  One JSON line per rate."""
    import torch
    from paper_2004_03054_amd import Context

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.max_batch is None:
        args.max_batch = 16 if args.resident else 1
    ctx = Context(0)
    jobs, tables, _ = build_batch_pool(ctx, args.jobs, args.scale)
    opts = [o for _, o in jobs]
    tbytes = [sum(int(t.numel()) for t in tabs) for tabs in tables]
    for rate in [float(x) for x in str(args.rate).split(",")]:
        rec = serve_record(args, tables, opts, tbytes, rate, args.duration, args.resident, args.max_batch,
                           args.workers, args.budget_gib, args.keep_s)
        out = {
            "metric": "p99 job latency (served)",
            "value": rec["served"]["p99_ms"],
            "unit": "ms",
            "n_gpus": 1,
            "steps": rec["served"]["jobs"],
            "warmup": 1,
            "ms_per_step": rec["served"]["p50_ms"],
            "higher_is_better": False,
            "scaling": "weak",
            "vs_baseline": None,
            "dtype": "u8",
            "data": "synthetic",
            "config": {"workload": f"served-poisson{rate:g}-pool{args.jobs}" +
                       ("" if args.scale == 1.0 else f"-scale{args.scale:g}"), **{k: v for k, v in rec.items()
                       if k not in ("served", "plain_per_job", "outputs_identical")}},
            "served": rec["served"],
            "plain_per_job": rec["plain_per_job"],
            "outputs_identical": rec["outputs_identical"],
        }
        print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
