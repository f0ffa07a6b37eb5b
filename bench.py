"""Benchmark: compaction input GB/s of one large compaction on one MI355X.

Workload: one upper table + 10 overlapping lower tables of ~64 MiB each
(~700 MiB of input), 16-byte Zipf(0.99) keys over 2^32, 1 KiB values, 2%
deletions, output not at the bottom level, 4 KiB blocks, restart interval 16,
10 bits/key Bloom filters, 64 MiB output tables.  The input tables are written
on the GPU by the library's own table writer from seeded synthetic entries and
stay resident in HBM; each timed step is one whole compaction (decode with
checksums, merge and drop, re-encode with index, filter and checksums), with
the output tables left in HBM.

The JSON line's `value` is input bytes / wall time of the timed steps.  Extra
fields: the end-to-end rate (host tables -> device -> host tables, PCIe
included), per-kernel times, the roofline of the dominant kernel, and the CPU
baseline (the plain oracle on this host, single thread).
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


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed counter summary,
    or None when it is missing or the kernel's sources changed since."""
    import hashlib
    import re
    try:
        text = open(TRAFFIC_FILE).read()
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
    kernel, e.g. merge rounds, summed)."""
    out = {}
    for k, v in ctx.stage_times():
        if k.startswith("kernel:"):
            name = k.split(":", 1)[1]
            out[name] = out.get(name, 0.0) + v
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--scale", type=float, default=1.0, help="table size scale (1.0 = 64 MiB tables)")
    ap.add_argument("--config", type=int, choices=[0, 1, 2], default=1,
                    help="plain mode: 0 = small (3 x 10k entries), 1 = large (11 x 64 MiB), 2 = variable-size keys "
                         "and values (7 x 32 MiB)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--e2e-steps", type=int, default=3)
    ap.add_argument("--copy-mib", type=int, default=1024, help="copy mode: bytes copied per launch (MiB)")
    ap.add_argument("--mode", choices=["plain", "batch", "serve", "copy", "coopsort"], default="plain",
                    help="plain: one large compaction (default); batch: many uneven jobs, "
                         "one batched pass vs one call per job; serve: Poisson arrivals through the "
                         "request loop vs plain per-job launches")
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
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (jobs are independent: "
              "several GPUs would each run their own jobs with no exchange)", file=sys.stderr)
        sys.exit(2)

    if args.mode == "batch":
        return batch_main(args)
    if args.mode == "serve":
        return serve_main(args)
    if args.mode == "copy":
        return copy_main(args)
    if args.mode == "coopsort":
        return coopsort_main(args)
    import numpy as np
    import torch
    from paper_2004_03054_amd import Context
    from workload import config0, config1, config2

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    t0 = time.time()
    job = {0: lambda: config0(), 1: lambda: config1(scale=args.scale), 2: lambda: config2(scale=args.scale)}[args.config]()
    log(f"[bench] generated {job.name}: {sum(r.n for r in job.runs)} entries in {time.time() - t0:.1f}s")
    ctx = Context(0)
    tables = device_tables(ctx, job)
    in_bytes = sum(int(t.numel()) for t in tables)
    log(f"[bench] {len(tables)} input tables on the device, {in_bytes / 2**20:.1f} MiB")
    opts = job.options()

    # warmup (also checks the result is well formed)
    res = None
    for _ in range(args.warmup):
        res = ctx.compact_dev(tables, opts, materialize=False)
        assert res.status == 0, (res.name, ctx.last_error())
    # timed steps: kernel-only (inputs resident in HBM, outputs left in HBM)
    ktimes = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    step_s = []
    for _ in range(args.steps):
        ts = time.perf_counter()
        res = ctx.compact_dev(tables, opts, materialize=False)  # returns after its stream is done
        step_s.append(time.perf_counter() - ts)
        ktimes.append(kernel_times(ctx))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t_start
    assert res.status == 0, (res.name, ctx.last_error())
    counters = ctx.counters()
    ms_step = dt * 1e3 / args.steps
    value = in_bytes * args.steps / dt / 1e9
    log(f"[bench] {args.steps} steps: {ms_step:.3f} ms/step, {value:.1f} GB/s input")

    # per-kernel average times over the timed steps
    names = sorted(set(k for kt in ktimes for k in kt))
    kavg = {n: float(np.mean([kt.get(n, 0.0) for kt in ktimes])) for n in names}
    # roofline of the dominant kernel from its algorithmic bytes:
    #   k_crc_data reads every input data block once (contents + trailer)
    #   k_encode reads every surviving value once and writes every output
    #   data block once (both approximated by the output data-block bytes)
    #   k_walk_emit writes one 36-byte entry record per input entry
    #   k_keys reads 16 bytes of record per entry, writes its key slot
    #   (8 * kw8 bytes) and 28 bytes of sort keys
    n_in = counters.get("entries_in", 0.0)
    kw8 = counters.get("kw8", 2.0)
    alg = {
        "k_crc_data": counters.get("data_bytes_in", 0.0),
        "k_encode": 2.0 * counters.get("data_bytes_out", 0.0),
        "k_walk_emit": 36.0 * n_in,
        "k_keys": n_in * (16.0 + 8.0 * kw8 + 28.0),
    }
    dom = max(alg, key=lambda k: kavg.get(k, 0.0))
    achieved = alg[dom] / (kavg[dom] * 1e-3) / 1e9 if kavg.get(dom) else 0.0
    roofline = {"kernel": dom, "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                # the committed counters were taken on the large workload only
                "traffic": measured_traffic(dom) if args.config == 1 and args.scale == 1.0 else None,
                "alg_bytes_per_launch": alg[dom], "avg_ms": round(kavg[dom], 4)}
    other = {k: {"avg_ms": round(kavg.get(k, 0.0), 4),
                 "gbps": round(alg[k] / (kavg[k] * 1e-3) / 1e9, 1) if kavg.get(k) else None}
             for k in alg}

    # end to end: host tables in, host tables out (PCIe both ways): the
    # library's C-ABI from host input buffers to its host result buffers
    # (the binding's copy of them into Python objects is left out)
    host_tables = [t.cpu().numpy().tobytes() for t in tables]
    e2e = None
    if args.e2e_steps > 0:
        r = ctx.compact(host_tables, opts, materialize=False)
        assert r.status == 0
        t1 = time.perf_counter()
        for _ in range(args.e2e_steps):
            r = ctx.compact(host_tables, opts, materialize=False)
            assert r.status == 0
        e2e_dt = time.perf_counter() - t1
        e2e = round(in_bytes * args.e2e_steps / e2e_dt / 1e9, 2)
        log(f"[bench] end to end: {e2e} GB/s")
    gpu_files = ctx.compact(host_tables, opts).files

    cpu = None
    if not args.no_cpu_baseline:
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

    out = {
        "metric": "compaction input GB/s",
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
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
    print(json.dumps(out), flush=True)
    ctx.close()


def batch_main(args):
    """Many independent uneven jobs: one batched pass over every stage vs one
    plain call per job, on the same device-resident inputs."""
    import numpy as np
    import torch
    from paper_2004_03054_amd import Context
    from workload import config3_job

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    ctx = Context(0)
    jobs, tables, in_bytes = [], [], 0
    t0 = time.time()
    for j in range(args.jobs):
        job = config3_job(j, scale=args.scale)
        tabs = device_tables(ctx, job)
        tables.append(tabs)
        jobs.append((job.name, job.options()))
        in_bytes += sum(int(t.numel()) for t in tabs)
        del job
        if (j + 1) % 16 == 0:
            log(f"[bench] {j + 1} jobs on the device, {in_bytes / 2**30:.2f} GiB, {time.time() - t0:.0f}s")
    log(f"[bench] {args.jobs} jobs, {in_bytes / 2**30:.2f} GiB of input tables resident")
    batch = [(tables[j], jobs[j][1]) for j in range(args.jobs)]
    # launch parameters from the autotuner, on a sample of the jobs
    tuned, tuned_ms = ctx.autotune(batch[:min(8, args.jobs)], device_inputs=True, rounds=1)
    log(f"[bench] autotuned launch parameters {tuned} ({tuned_ms:.1f} ms on the sample)")
    # verification pass (outside timing): batched outputs == per-job outputs
    res_b = ctx.compact_batch(batch, device_inputs=True, materialize=fingerprint)
    fp_b = [r.files for r in res_b]
    status_b = [r.status for r in res_b]
    del res_b
    fp_p = []
    for j in range(args.jobs):
        r = ctx.compact_dev(tables[j], jobs[j][1], materialize=fingerprint)
        fp_p.append(r.files)
        assert r.status == 0 and status_b[j] == 0, (j, r.name, ctx.last_error())
    same = fp_p == fp_b
    log(f"[bench] batched outputs identical to per-job outputs: {same}")
    torch.cuda.synchronize()
    # timed: plain loop, then batched
    steps = max(1, args.steps)
    tp = time.perf_counter()
    for _ in range(steps):
        for j in range(args.jobs):
            ctx.compact_dev(tables[j], jobs[j][1], materialize=False)
    torch.cuda.synchronize()
    plain_s = (time.perf_counter() - tp) / steps
    tb = time.perf_counter()
    for _ in range(steps):
        out = ctx.compact_batch(batch, device_inputs=True, materialize=False)
    torch.cuda.synchronize()
    batch_s = (time.perf_counter() - tb) / steps
    assert all(r.status == 0 for r in out)
    value = in_bytes / batch_s / 1e9
    plain = in_bytes / plain_s / 1e9
    log(f"[bench] batched {batch_s * 1e3:.1f} ms ({value:.1f} GB/s), plain loop {plain_s * 1e3:.1f} ms "
        f"({plain:.1f} GB/s)")
    kt = kernel_times(ctx)
    cpu = None
    threads = args.oracle_threads or min(16, os.cpu_count() or 1)
    n_oracle = min(args.oracle_jobs or threads, len(tables))
    if n_oracle > 0:
        # the oracle on the host cores: independent jobs of the batch on
        # `threads` threads at once (the oracle is C called through ctypes,
        # which runs without the interpreter lock), aggregate input GB/s
        from concurrent.futures import ThreadPoolExecutor
        import oracle
        from workload import config3_job as mk
        jobs_o = [mk(j, scale=args.scale) for j in range(n_oracle)]
        ins_o = [oracle.build_input_tables(job) for job in jobs_o]

        def run_one(k):
            return oracle.compact(ins_o[k], jobs_o[k].options())

        t2 = time.perf_counter()
        with ThreadPoolExecutor(max_workers=threads) as ex:
            refs = list(ex.map(run_one, range(n_oracle)))
        tot_t = time.perf_counter() - t2
        tot_b = sum(sum(len(x) for x in ins) for ins in ins_o)
        exact = True
        for j in range(n_oracle):
            host = [t.cpu().numpy().tobytes() for t in tables[j]]
            r = ctx.compact(host, jobs_o[j].options())
            exact = exact and ins_o[j] == host and refs[j].status == 0 and refs[j].files == r.files
        cpu = {"value": round(tot_b / tot_t / 1e9, 4), "unit": "GB/s", "cores": min(threads, n_oracle),
               "kind": "oracle",
               "sample": f"jobs 0..{n_oracle - 1} of the batch ({tot_b / 2**20:.0f} MiB) on "
                         f"{min(threads, n_oracle)} threads, {tot_t:.1f} s wall",
               "bit_exact": bool(exact), "host": host_info()}
        log(f"[bench] oracle: {n_oracle} jobs on {min(threads, n_oracle)} threads in {tot_t:.1f}s, "
            f"bit-exact {exact}")
    out = {
        "metric": "compaction input GB/s (batched)",
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": 1,
        "ms_per_step": round(batch_s * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": f"batch-{args.jobs}-jobs" + ("" if args.scale == 1.0 else f"-scale{args.scale:g}"),
                   "jobs": args.jobs, "input_bytes": in_bytes, "inputs_resident": "hbm", "outputs": "hbm"},
        "plain_loop_gbps": round(plain, 2),
        "batched_over_plain": round(plain_s / batch_s, 3),
        "outputs_identical": bool(same),
        "launch_params": tuned,
        "kernel_ms": {k: round(v, 4) for k, v in kt.items()},
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
    from workload import config1

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    job = config1(scale=args.scale)
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


def serve_main(args):
    """Poisson arrivals of jobs drawn from the batch workload's job mixture,
    through the request loop (admission under an HBM budget, batched passes
    on two workers) and through plain per-job launches (one job at a time),
    on the same trace.  Latency = completion (outputs in host memory; in HBM
    with --resident) minus
    arrival."""
    import numpy as np
    import torch
    from paper_2004_03054_amd import Context, Server
    from workload import config3_job

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.max_batch is None:
        args.max_batch = 16 if args.resident else 1
    ctx = Context(0)
    tables, opts, tbytes = [], [], []
    for j in range(args.jobs):
        job = config3_job(j, scale=args.scale)
        tabs = device_tables(ctx, job)
        tables.append(tabs)
        opts.append(job.options())
        tbytes.append(sum(int(t.numel()) for t in tabs))
    log(f"[bench] pool of {args.jobs} jobs, {sum(tbytes) / 2**30:.2f} GiB resident")
    for rate in [float(x) for x in str(args.rate).split(",")]:
        rng = np.random.default_rng(0x5E5E)
        n = max(1, int(rate * args.duration))
        arrivals = np.cumsum(rng.exponential(1.0 / rate, n)).tolist()
        picks = rng.integers(0, args.jobs, n).tolist()
        budget = int(args.budget_gib * 2**30)
        sub = None
        if args.resident:
            # with probability 1/2 a request's first lower input is replaced by the
            # output tables of a request that arrived at least 1 s earlier
            # (from the last --keep-s seconds of arrivals, so that older outputs can be freed)
            sub = []
            for k, at in enumerate(arrivals):
                early = [q for q in range(k) if at - args.keep_s <= arrivals[q] <= at - 1.0]
                sub.append(int(rng.choice(early)) if early and rng.random() < 0.5 else None)
            log(f"[bench] {sum(x is not None for x in sub)} of {n} requests read earlier outputs kept in HBM")
        results = {}
        for name, kw in (("served", dict(max_batch_jobs=args.max_batch, workers=args.workers)),
                         ("plain", dict(max_batch_jobs=1, workers=1))):
            srv = Server(0, hbm_budget=budget, host_outputs=not args.resident, **kw)
            # warm the workers' buffers on the largest job
            big = int(np.argmax(tbytes))
            srv.poll(srv.submit(tables[big], opts[big]))
            out, span = run_trace(srv, arrivals, picks, tables, opts, tbytes, sub, args.keep_s)
            st = srv.stats()
            srv.close()
            lat = np.array([o[0] for o in out])
            warm = np.array(arrivals) >= min(2.0, args.duration * 0.2)  # drop the start-up interval
            lw = lat[warm] if warm.any() else lat
            results[name] = dict(p50_ms=round(float(np.percentile(lw, 50)), 3), p99_ms=round(float(np.percentile(lw, 99)), 3),
                                 gbps=round(sum(o[1] for o in out) / span / 1e9, 3), jobs=n, batches=st["batches"],
                                 max_batch=st["max_batch"], peak_admitted_gib=round(st["peak_admitted"] / 2**30, 2),
                                 digests=[o[2] for o in out])
            log(f"[bench] {name}: p50 {results[name]['p50_ms']} ms, p99 {results[name]['p99_ms']} ms, "
                f"{results[name]['gbps']} GB/s, {st['batches']} passes")
            slow = np.argsort(lat)[-5:][::-1]
            log(f"[bench] {name} slowest (request, arrival s, input MiB, ms): " +
                ", ".join(f"({int(q)}, {arrivals[q]:.2f}, {out[q][1] / 2**20:.0f}, {lat[q]:.1f})" for q in slow))
        same = results["served"].pop("digests") == results["plain"].pop("digests")
        log(f"[bench] every served job's outputs identical to its plain run: {same}")
        out = {
            "metric": "p99 job latency (served)",
            "value": results["served"]["p99_ms"],
            "unit": "ms",
            "n_gpus": 1,
            "steps": n,
            "warmup": 1,
            "ms_per_step": results["served"]["p50_ms"],
            "higher_is_better": False,
            "scaling": "weak",
            "vs_baseline": None,
            "dtype": "u8",
            "data": "synthetic",
            "config": {"workload": f"served-poisson{rate:g}-pool{args.jobs}" +
                       ("" if args.scale == 1.0 else f"-scale{args.scale:g}"),
                       "rate_per_s": rate, "duration_s": args.duration, "hbm_budget_gib": args.budget_gib,
                       "max_batch_jobs": args.max_batch, "workers": args.workers,
                       "outputs": "hbm" if args.resident else "host",
                       "resident_inputs": bool(args.resident),
                   **({"keep_s": args.keep_s} if args.resident else {})},
            "served": results["served"],
            "plain_per_job": results["plain"],
            "outputs_identical": bool(same),
        }
        print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
