#!/usr/bin/env python3
"""Benchmark of the ttx hot path on one MI355X.

Workload (one "step"): the 36 paper-shaped transpositions of about 200 MiB
per tensor -- 4D, 5D and 6D, FP32 and FP64, beta = 0.7 and beta = 0 with
alpha = 1.3 -- each through its plan with its size-specialised kernel, on
its own device buffers (14 GiB in all, so no tensor is still cached in the
256 MiB Infinity Cache when its turn comes).  The reported value is the
whole step's algorithmic traffic (2S bytes for beta = 0, 3S otherwise, S the
bytes of the transposed tensor; Sec. 3, Eqn. 2) divided by its wall time.

Also measured: every case against a hipMemcpy device-to-device ceiling, the
dominant kernel against the HBM roofline (8 TB/s), the CPU oracle on the
host (which also checks every element of every case's GPU output), the
leading-dimension, awkward and literal shapes, the 512-problem batch, the
served trace, the complex, mixed-precision and packing cases, and three
tensor contractions by transpose-transpose-GEMM-transpose (whole, panel
GEMM alone, and torch's tensordot on the same tensors).  The printed JSON
line holds the summary; the per-case detail goes to ``--detail-out``.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import glob
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBPS = 8000.0          # MI355X HBM3E, published
TABLE = os.path.join(ROOT, "paper_1607_01249_amd", "tune", "gfx950.txt")
# submitting threads of the served runs (clients sharing one server)
CLIENTS = 4
# device slots (micro-batches in flight) of the served runs
SLOTS = 8
TRAFFIC = os.path.join(ROOT, "profiles", "traffic_counters.json")
# the per-call kernels' sources (their code, without comments, keys the counter traffic)
KERNEL_SOURCES = (["device_types.h", "tile_kernels.h", "menu.h", "registry.h", "moved_launch.h",
                   "staged_launch.h", "dispatch.hip", "jit.cpp"] +
                  sorted(os.path.basename(f) for f in glob.glob(os.path.join(
                      os.path.dirname(os.path.abspath(__file__)), "paper_1607_01249_amd", "csrc",
                      "kernels_*.hip"))))
METRIC = "achieved HBM GB/s (% of D2D-copy peak) per perm; batched p50/p99 latency vs per-call"


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_source_hash():
    """Hash of the kernel sources with comments and blank lines left out (a
    comment edit does not invalidate measured counters)."""
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1607_01249_amd", "csrc", name)) as f:
            for line in f:
                code = line.split("//", 1)[0].rstrip()
                if code:
                    h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def parse_args():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--tune-candidates", type=int, default=100,
                    help="candidates timed per shape missing from the tune table")
    ap.add_argument("--retune", action="store_true", help="ignore the shipped tune table")
    ap.add_argument("--save-table", default=None, help="write the tune table here")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--dominant-out", default=None,
                    help="also write the dominant kernel's name and launch figures to this JSON file")
    ap.add_argument("--literal", action="store_true",
                    help="add the literal (160,160,160,160) FP32/FP64 shapes to the step")
    ap.add_argument("--no-batched", action="store_true", help="skip the 512-problem batched comparison")
    ap.add_argument("--generic", action="store_true",
                    help="time the step through ttx_transpose with the generic kernels (no run-time compilation)")
    ap.add_argument("--no-specialised", action="store_true",
                    help="skip the comparison with size-specialised (run-time compiled) kernels")
    ap.add_argument("--no-served", action="store_true", help="skip the serving comparison")
    ap.add_argument("--no-side", action="store_true",
                    help="skip the side shapes (leading dimensions, awkward extents, literal 160^4 and 24^6)")
    ap.add_argument("--detail-out", default=os.path.join("gpurun_out", "bench_detail.json"),
                    help="the per-case detail (JSON); the printed line holds the summary")
    ap.add_argument("--no-types", action="store_true",
                    help="skip the complex (c, z) and mixed-precision (sd, ds, cz, zc) cases")
    ap.add_argument("--no-contraction", action="store_true",
                    help="skip the transpose-transpose-GEMM-transpose contractions")
    ap.add_argument("--only-contraction", action="store_true",
                    help="for rocprofv3: only the contractions (after the ceilings), then exit")
    ap.add_argument("--serve-seconds", type=float, default=10.0)
    ap.add_argument("--serve-rate", type=float, default=20000.0, help="Poisson arrival rate (req/s)")
    ap.add_argument("--profile-run", action="store_true",
                    help="short run for rocprofv3: no tuning, 1 warm-up, 2 steps, no CPU leg")
    ap.add_argument("--profile-batched", action="store_true",
                    help="for rocprofv3: only the 512-problem batched comparison, untuned, 5 replays")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_DB", "WRITE_DB"),
                    help="summarise two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE) of this "
                         "script into profiles/traffic_counters.json and exit")
    ap.add_argument("--traffic-out", default=None,
                    help="where --traffic-from writes (default profiles/traffic_counters.json)")
    ap.add_argument("--summarize-counters", metavar="DB",
                    help="print a markdown table of the SQ counters (waves, LDS instructions, LDS bank "
                         "conflict cycles) and the register, LDS and scratch budgets of each ttx kernel "
                         "in a rocprofv3 --pmc database, and exit")
    ap.add_argument("--summarize-trace", metavar="DB",
                    help="print the kernel statistics of a rocprofv3 --kernel-trace --stats run")
    return ap.parse_args()


# ---------------------------------------------------------------------------------------
def make_cases(literal):
    import workloads
    cases = workloads.large_cases()
    if literal:
        for dtype in (workloads.F32, workloads.F64):
            for perm in [(3, 2, 1, 0), (2, 0, 3, 1)]:
                cases.append(dict(name="literal160_%s_p%s_b0.7" % ("f32" if dtype == workloads.F32 else "f64",
                                                                    "".join(map(str, perm))),
                                  dtype=dtype, size=workloads.LITERAL_4D, perm=perm, alpha=1.3,
                                  beta=0.7, seed_a=3000, seed_b=3001))
    for c in cases:
        c["elements"] = workloads.elements(c["size"])
        S = c["elements"] * c["dtype"].itemsize
        c["bytes"] = (2 if c["beta"] == 0 else 3) * S
    return cases


def fill_uniform(torch, t, seed):
    """Seeded uniform [-1, 1) values generated on the device."""
    g = torch.Generator(device=t.device)
    g.manual_seed(int(seed))
    t.uniform_(-1.0, 1.0, generator=g)


def time_events(torch, fn, reps, flush=None):
    """Minimum and median of `reps` runs of fn() bracketed by events (flush before each)."""
    times = []
    for _ in range(reps):
        if flush is not None:
            flush()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        e1.synchronize()
        times.append(e0.elapsed_time(e1) * 1e-3)
    return min(times), float(np.median(times))


def hip_runtime():
    """The HIP runtime torch loaded (so that streams are shared)."""
    import ctypes
    maps = open("/proc/self/maps").read().splitlines()
    paths = sorted({l.split()[-1] for l in maps if "libamdhip64" in l})
    L = ctypes.CDLL(paths[0] if paths else "libamdhip64.so")
    L.hipMemcpyAsync.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int,
                                 ctypes.c_void_p]
    L.hipMemcpyAsync.restype = ctypes.c_int
    L.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    L.hipMemcpy.restype = ctypes.c_int
    return L


def measure_ceilings(torch, ttx):
    """hipMemcpy D2D (the metric's denominator), a 16-byte copy kernel and an
    unfused axpby (the SAXPY peak of Sec. 3) on 1 GiB buffers.  Four buffer
    pairs are used in rotation, so that each run streams data the previous
    runs have pushed out of the 256 MiB Infinity Cache (no flush kernel runs
    in between whose dirty lines would be written back during the run)."""
    nbytes = 1 << 30
    pairs = []
    for i in range(4):
        src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        fill_uniform(torch, src, 1 + i)
        fill_uniform(torch, dst, 11 + i)
        pairs.append((src, dst))
    torch.cuda.synchronize()
    hip = hip_runtime()
    stream = torch.cuda.current_stream().cuda_stream
    state = {"i": 0}

    def nxt():
        state["i"] = (state["i"] + 1) % len(pairs)
        return pairs[state["i"]]

    def d2d():
        src, dst = nxt()
        rc = hip.hipMemcpyAsync(dst.data_ptr(), src.data_ptr(), nbytes, 3, stream)
        assert rc == 0, rc

    def copyk():
        src, dst = nxt()
        ttx.ttx_copy_kernel(src.data_ptr(), dst.data_ptr(), nbytes, stream)

    def axpby():
        src, dst = nxt()
        ttx.ttx_axpby_kernel(ttx.F32, nbytes // 4, 1.3, src.data_ptr(), 0.7, dst.data_ptr(), stream)

    out = {}
    for name, fn, moved in [("hipMemcpy_d2d", d2d, 2 * nbytes), ("copy_kernel", copyk, 2 * nbytes),
                            ("axpby_f32", axpby, 3 * nbytes)]:
        for _ in range(4):
            fn()
        tmin, tmed = time_events(torch, fn, 12)
        out[name] = dict(GBps=round(moved / tmin / 1e9, 1), GBps_median=round(moved / tmed / 1e9, 1),
                         bytes=moved)
    del pairs
    return out


def _ulp_diff(x, y):
    """Largest distance in units in the last place between two float arrays of
    one dtype (complex arrays compared part by part); NaNs of either sign
    count as equal to each other."""
    if x.dtype.kind == "c":
        x = x.view(np.float32 if x.dtype == np.complex64 else np.float64)
        y = y.view(x.dtype)
    it = np.int32 if x.dtype == np.float32 else np.int64
    xi, yi = x.view(it).astype(np.int64), y.view(it).astype(np.int64)
    # map the sign-magnitude bit patterns to one ordered integer line
    lo = np.iinfo(it).min
    xo = np.where(xi < 0, lo - xi, xi)
    yo = np.where(yi < 0, lo - yi, yi)
    d = np.abs(xo - yo)
    both_nan = np.isnan(x) & np.isnan(y)
    d[both_nan] = 0
    return int(d.max()) if d.size else 0


def host_cpu_info():
    """The host's core counts and processor model (for the CPU baseline)."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return dict(logical_cpus=os.cpu_count(), usable_cpus=usable, model=model,
                omp_num_threads=os.environ.get("OMP_NUM_THREADS"))


def cpu_baseline(torch, ttx, cases, stream, one_thread_every=3):
    """The oracle (plain C loop nest, OpenMP over the outermost B index) on the
    host cores, on every case of the step, timed (min of 3 runs per case) on
    the inputs of one more GPU call of that case copied from the device; the
    GPU's output of that call is compared with the oracle's first run element
    by element.  Then a 1-thread run of every ``one_thread_every``-th case."""
    os.environ.setdefault("OMP_PROC_BIND", "close")
    os.environ.setdefault("OMP_PLACES", "cores")
    import oracle
    t_start = time.time()
    per_case, total_bytes, total_t = [], 0, 0.0
    mismatched, max_ulp, compared = 0, 0, 0
    for c in cases:
        A = c["A"].cpu().numpy()
        B0 = c["B"].cpu().numpy()                      # B before the call
        ttx.ttx_plan_execute(c["plan"], c["alpha"], c["A"].data_ptr(), c["beta"], c["B"].data_ptr(), stream)
        torch.cuda.synchronize()
        G = c["B"].cpu().numpy()                       # the GPU's result
        best = None
        for r in range(3):
            B = B0.copy()
            t0 = time.perf_counter()
            st = oracle.transpose(c["perm"], c["size"], c["alpha"], A, c["beta"], B)
            dt = time.perf_counter() - t0
            assert st == 0, st
            best = dt if best is None else min(best, dt)
            if r == 0:
                bits = np.int64 if B.itemsize == 8 else np.int32
                diff = int(np.count_nonzero(B.view(bits) != G.view(bits)))
                mismatched += diff
                compared += B.size
                if diff:
                    max_ulp = max(max_ulp, _ulp_diff(B, G))
        total_bytes += c["bytes"]
        total_t += best
        per_case.append(dict(case=c["name"], GBps=round(c["bytes"] / best / 1e9, 2), s=round(best, 4),
                             differing_elements=diff))
        del A, B0, G, B
    threads = oracle.threads()
    # the same loop nest on one thread, on a sample of the cases
    one = None
    if one_thread_every:
        import workloads
        prev = oracle.set_threads(1)
        b1, t1, names = 0, 0.0, []
        try:
            for c in cases[::one_thread_every]:
                A = workloads.uniform(c["elements"], c["dtype"], c["seed_a"])
                B = workloads.uniform(c["elements"], c["dtype"], c["seed_b"])
                t0 = time.perf_counter()
                assert oracle.transpose(c["perm"], c["size"], c["alpha"], A, c["beta"], B) == 0
                t1 += time.perf_counter() - t0
                b1 += c["bytes"]
                names.append(c["name"])
                del A, B
        finally:
            oracle.set_threads(threads if threads >= 1 else prev)
        one = dict(value=round(b1 / t1 / 1e9, 3), unit="GB/s", cores=1,
                   sample="%d cases (every %d-th of the step), 1 run each" % (len(names), one_thread_every))
    verification = dict(cases=len(cases), elements_compared=compared, differing_elements=mismatched,
                        max_ulp=max_ulp, verified=bool(max_ulp <= 1),
                        how="every element of every case's GPU output against the oracle on the same inputs")
    return dict(value=round(total_bytes / total_t / 1e9, 3), unit="GB/s", cores=threads, kind="oracle",
                sample="all %d cases of the step, min of 3 runs each, inputs of one GPU call copied from the "
                       "device" % len(cases),
                one_thread=one, host=host_cpu_info(), seconds=round(time.time() - t_start, 1),
                per_case=per_case), verification


def _rocpd(path):
    import sqlite3
    files = [path] if path.endswith(".db") else glob.glob(os.path.join(path, "**", "*.db"), recursive=True)
    assert files, "no rocpd database under %s" % path
    return [sqlite3.connect(f) for f in files]


def _short_kernel(name):
    """'void ttx::k_moved<float, false, 64, 64, 4, 4>(ttx::TileArgs<float>)' -> 'k_moved<...>'."""
    name = name.replace("void ", "").replace("ttx::", "")
    depth, out = 0, ""
    for ch in name:
        if ch == "(" and depth == 0:
            break
        depth += ch == "<"
        depth -= ch == ">"
        out += ch
    return out


def traffic_from(fetch_path, write_path, out_path=None):
    """Per-dispatch FETCH_SIZE and WRITE_SIZE (KiB) of every ttx kernel from two
    rocprofv3 --pmc runs of bench.py, each scaled by what the same counter
    reads for the 1 GiB copy kernel (1 GiB read, 1 GiB written)."""
    res = {}
    for counter, path in (("FETCH_SIZE", fetch_path), ("WRITE_SIZE", write_path)):
        per = {}
        for db in _rocpd(path):
            for name, cname, val in db.execute("select name, counter_name, counter_value from pmc_events"):
                if cname == counter:
                    per.setdefault(_short_kernel(name), []).append(float(val))
        copy = per.get("k_copy16")
        assert copy, "copy kernel missing from the %s run" % counter
        scale = (1 << 30) / (float(np.median(copy)) * 1024.0)
        res[counter] = dict(scale=scale, copy_kib=float(np.median(copy)),
                            kernels={k: dict(kib=float(np.mean(v)), dispatches=len(v))
                                     for k, v in per.items() if k.startswith(("k_", "ttx_jit_"))})
    table = {}
    for k, f in res["FETCH_SIZE"]["kernels"].items():
        w = res["WRITE_SIZE"]["kernels"].get(k)
        if w is None:
            continue
        fb = f["kib"] * 1024 * res["FETCH_SIZE"]["scale"]
        wb = w["kib"] * 1024 * res["WRITE_SIZE"]["scale"]
        table[k] = dict(fetch_bytes=round(fb), write_bytes=round(wb), traffic_bytes=round(fb + wb),
                        dispatches=f["dispatches"])
    out = dict(source_hash=kernel_source_hash(),
               scale=dict(FETCH_SIZE=res["FETCH_SIZE"]["scale"], WRITE_SIZE=res["WRITE_SIZE"]["scale"]),
               copy_kernel_kib=dict(FETCH_SIZE=res["FETCH_SIZE"]["copy_kib"],
                                    WRITE_SIZE=res["WRITE_SIZE"]["copy_kib"]),
               kernels=table)
    with open(out_path or TRAFFIC, "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
    print(json.dumps(out, sort_keys=True))


def summarize_counters(path):
    """Per ttx kernel of a rocprofv3 --pmc database: the mean of each SQ counter
    per dispatch, LDS bank-conflict cycles per LDS instruction, and the
    kernel's VGPRs, LDS bytes and scratch bytes per lane with the waves per
    SIMD they allow (512 VGPRs per SIMD lane, 160 KiB of LDS per CU, 4 SIMDs
    and at most 8 waves each)."""
    counters, budget = {}, {}
    for db in _rocpd(path):
        for name, cname, val in db.execute("select name, counter_name, counter_value from pmc_events"):
            k = _short_kernel(name) if "ttx::" in name else name
            if k.startswith(("ttx_jit_", "k_")):
                counters.setdefault(k, {}).setdefault(cname, []).append(float(val))
        for name, vgpr, lds, priv in db.execute(
                "select kernel_name, arch_vgpr_count, group_segment_size, private_segment_size from kernel_symbols"):
            name = name[:-3] if name.endswith(".kd") else name   # the kernel descriptor's symbol
            k = _short_kernel(name) if "ttx::" in name else name
            budget[k] = (int(vgpr), int(lds), int(priv))
    names = sorted({c for v in counters.values() for c in v})
    lines = ["| kernel | " + " | ".join(names) + " | conflict cycles / LDS instr | VGPRs | LDS B | scratch B/lane |"
             " waves/SIMD (VGPR) |", "|---|" + "---|" * (len(names) + 5)]
    for k in sorted(counters):
        mean = {c: float(np.mean(v)) for c, v in counters[k].items()}
        ratio = (mean.get("SQ_LDS_BANK_CONFLICT", 0.0) / mean["SQ_INSTS_LDS"]) if mean.get("SQ_INSTS_LDS") else 0.0
        vgpr, lds, priv = budget.get(k, (0, 0, 0))
        waves = min(8, 512 // max(8, -(-vgpr // 8) * 8)) if vgpr else 0
        lines.append("| %s | %s | %.2f | %d | %d | %d | %d |" % (
            k, " | ".join("%.0f" % mean.get(c, float("nan")) for c in names), ratio, vgpr, lds, priv, waves))
    print("\n".join(lines))


def summarize_trace(path, top=25):
    """Markdown table of the kernel statistics in a rocprofv3 --kernel-trace --stats database."""
    rows = {}
    for db in _rocpd(path):
        for name, calls, total, avg in db.execute(
                "select name, total_calls, total_duration, average from top_kernels"):
            k = _short_kernel(name) if "ttx::" in name else name[:60]
            r = rows.setdefault(k, [0, 0.0])
            r[0] += calls
            r[1] += total
    total_all = sum(r[1] for r in rows.values())
    lines = ["| kernel | calls | total us | average us | % |", "|---|---|---|---|---|"]
    for k, (calls, total) in sorted(rows.items(), key=lambda kv: -kv[1][1])[:top]:
        lines.append("| %s | %d | %.1f | %.2f | %.1f |" % (k, calls, total, total / calls,
                                                          100 * total / total_all))
    print("\n".join(lines))


def _pct(v, q):
    return float(np.percentile(np.asarray(v), q)) if len(v) else None


def bench_batched(torch, ttx, reps=20, tune=True):
    """The 512 uneven transpositions: per-call loop vs one graph-captured
    persistent launch (after per-shape tuning)."""
    import workloads
    probs = workloads.batched_problems()
    stream = torch.cuda.current_stream().cuda_stream
    tens, qs, nbytes = [], [], 0
    for i, p in enumerate(probs):
        n = workloads.elements(p["size"])
        tdt = torch.float32 if p["dtype"].itemsize == 4 else torch.float64
        A = torch.empty(n, dtype=tdt, device="cuda")
        B = torch.empty(n, dtype=tdt, device="cuda")
        fill_uniform(torch, A, 5000 + 2 * i)
        fill_uniform(torch, B, 5001 + 2 * i)
        tens.append((A, B))
        qs.append(ttx.make_problem(ttx.F32 if tdt == torch.float32 else ttx.F64, p["perm"], p["size"],
                                   p["alpha"], A.data_ptr(), p["beta"], B.data_ptr()))
        nbytes += n * p["dtype"].itemsize * (2 if p["beta"] == 0 else 3)
    torch.cuda.synchronize()

    def per_call():
        for q in qs:
            ttx.ttx_transpose(q.dtype, q.n, list(q.perm[:q.n]), list(q.size[:q.n]), None, None, q.alpha,
                              q.A, q.beta, q.B, stream)

    per_call()
    per_call()
    pc_min, pc_med = time_events(torch, per_call, reps)
    lat_pc = []
    for q in qs:   # one call at a time, synchronised: the per-call latency
        t0 = time.perf_counter()
        ttx.ttx_transpose(q.dtype, q.n, list(q.perm[:q.n]), list(q.size[:q.n]), None, None, q.alpha,
                          q.A, q.beta, q.B, stream)
        torch.cuda.current_stream().synchronize()
        lat_pc.append((time.perf_counter() - t0) * 1e6)
    h = ttx.ttx_batch_create(qs)
    t0 = time.time()
    if tune:
        ttx.ttx_batch_tune(h, 8, 2)
    tune_s = time.time() - t0
    info = ttx.ttx_batch_get_info(h)
    run = lambda: ttx.ttx_batch_execute(h, stream)
    run()
    run()
    times = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        run()
        e1.record()
        e1.synchronize()
        times.append(e0.elapsed_time(e1) * 1e-3)
    ttx.ttx_batch_destroy(h)
    del tens
    b_min, b_med = min(times), float(np.median(times))
    return dict(problems=len(qs), algorithmic_bytes=nbytes,
                per_call=dict(GBps=round(nbytes / pc_med / 1e9, 1), ms=round(pc_med * 1e3, 3),
                              launches=len(qs), call_latency_p50_us=round(_pct(lat_pc, 50), 1),
                              call_latency_p99_us=round(_pct(lat_pc, 99), 1)),
                batched=dict(GBps=round(nbytes / b_med / 1e9, 1), ms=round(b_med * 1e3, 3),
                             makespan_p50_ms=round(_pct(times, 50) * 1e3, 3),
                             makespan_p99_ms=round(_pct(times, 99) * 1e3, 3),
                             grid=info["grid"], tiles=info["total_tiles"], chunks=info["chunks"],
                             variants=info["variants_used"], tuned=info["tuned"],
                             tune_seconds=round(tune_s, 1), launch="1 persistent kernel per hipGraph replay"),
                speedup=round(pc_med / b_med, 2))


def bench_specialised(torch, ttx, cases, d2d, stream, steps=10, reps=5):
    """The step's cases through plans with their generic kernels, with
    size-specialised kernels (compiled at run time with the sizes as
    constants) for every case, and with specialised kernels where timing
    chose them (ttx_plan_specialise with reps > 0): alternating whole steps
    (every launch sees the same cache state as in the headline step), events
    around each launch, medians over the steps; and the compile time."""
    n = len(cases)
    plans = {"generic": [], "specialised": [], "tuned": []}
    compile_s, kept = 0.0, 0
    for c in cases:
        z = c["beta"] == 0
        for k in plans:
            plans[k].append(ttx.ttx_plan_create(c["code"], c["perm"], c["size"]))
        t0 = time.perf_counter()
        ttx.ttx_plan_specialise(plans["specialised"][-1], z)
        compile_s += time.perf_counter() - t0
        kept += ttx.ttx_plan_specialise(plans["tuned"][-1], z, reps=reps)
    try:
        def run(ps, ev=None):
            for i, c in enumerate(cases):
                if ev is not None:
                    ev[i].record()
                ttx.ttx_plan_execute(ps[i], c["alpha"], c["A"].data_ptr(), c["beta"], c["B"].data_ptr(), stream)
            if ev is not None:
                ev[n].record()

        for ps in plans.values():
            run(ps)
        ev = {k: [[torch.cuda.Event(enable_timing=True) for _ in range(n + 1)] for _ in range(steps)]
              for k in plans}
        for s in range(steps):
            for k, ps in plans.items():
                run(ps, ev[k][s])
        torch.cuda.synchronize()
        chosen = [ttx.ttx_plan_describe(p)["specialised"][int(c["beta"] == 0)] for p, c in zip(plans["tuned"], cases)]
    finally:
        for ps in plans.values():
            for p in ps:
                ttx.ttx_plan_destroy(p)
    med = {k: [float(np.median([e[s][i].elapsed_time(e[s][i + 1]) for s in range(steps)])) * 1e-3
               for i in range(n)] for k, e in ev.items()}
    step = {k: float(np.median([e[s][0].elapsed_time(e[s][n]) for s in range(steps)])) * 1e-3
            for k, e in ev.items()}
    step_bytes = sum(c["bytes"] for c in cases)
    out = []
    for i, c in enumerate(cases):
        g, s, t = med["generic"][i], med["specialised"][i], med["tuned"][i]
        out.append(dict(case=c["name"], generic_us=round(g * 1e6, 1), specialised_us=round(s * 1e6, 1),
                        speedup=round(g / s, 3), chosen=bool(chosen[i]), tuned_us=round(t * 1e6, 1)))
    sp_all = [o["speedup"] for o in out]
    return dict({"step_GBps_" + k: round(step_bytes / v / 1e9, 1) for k, v in step.items()},
                speedup_min=min(sp_all), speedup_median=float(np.median(sp_all)), speedup_max=max(sp_all),
                kept_by_timing=kept, compile_seconds=round(compile_s, 2), steps=steps, timing_reps=reps,
                note="alternating whole steps through plans; step = events from the first launch to the last",
                per_case=out)


def bench_types(torch, ttx, d2d, stream, tune_candidates, reps=10, profile=False, specialise=True):
    """Transpositions of the other element types through plans with their
    size-specialised kernels (as the main step runs its cases; generic
    kernels with specialise=False): complex (c and z, complex alpha and beta)
    about 200 MiB per tensor, and mixed precision (sd, ds, cz, zc), beta != 0,
    one case resident at a time: the median time of `reps` launches per case
    (bytes: read A, read and write B).
    Launches rotate over three (A, B) pairs so that each one starts with the
    data of the two before it in the 256 MiB Infinity Cache, not its own."""
    import workloads
    out = []
    tdt = {workloads.F32: torch.float32, workloads.F64: torch.float64,
           workloads.C32: torch.complex64, workloads.C64: torch.complex128}
    tcode = {workloads.F32: ttx.F32, workloads.F64: ttx.F64, workloads.C32: ttx.C32,
             workloads.C64: ttx.C64}
    tuned = 0
    for c in workloads.complex_cases() + workloads.mixed_cases():
        n = workloads.elements(c["size"])
        code = ttx.CODE_OF[(tcode[c["dtype_a"]], tcode[c["dtype"]])]
        plan = ttx.ttx_plan_create(code, c["perm"], c["size"])
        if not ttx.ttx_plan_describe(plan)["config_from_table"][0]:
            if profile:
                raise SystemExit("--profile-run needs every case in the tune table (%s)" % c["name"])
            log("tuning %s" % c["name"])
            ttx.ttx_tune(code, c["perm"], c["size"], beta_is_zero=False,
                         max_candidates=tune_candidates, reps=3)
            ttx.ttx_plan_destroy(plan)
            plan = ttx.ttx_plan_create(code, c["perm"], c["size"])
            tuned += 1
        if specialise:
            try:
                ttx.ttx_plan_specialise(plan, False)
            except ttx.TTXError as e:
                log("specialisation failed for %s (%s): generic kernel" % (c["name"], e))
        pairs = []
        real = lambda t: torch.view_as_real(t) if t.is_complex() else t
        for k in range(3):
            A = torch.empty(n, dtype=tdt[c["dtype_a"]], device="cuda")
            B = torch.empty(n, dtype=tdt[c["dtype"]], device="cuda")
            fill_uniform(torch, real(A), c["seed_a"] + 100 * k)
            fill_uniform(torch, real(B), c["seed_b"] + 100 * k)
            pairs.append((A, B))
        kernel = ttx.ttx_plan_kernel_name(plan, 1.0, pairs[0][0].data_ptr(), pairs[0][1].data_ptr())
        state = {"i": 0}

        def run():
            state["i"] = (state["i"] + 1) % len(pairs)
            A, B = pairs[state["i"]]
            ttx.ttx_plan_execute_c(plan, c["alpha"], A.data_ptr(), c["beta"], B.data_ptr(),
                                   B.data_ptr(), stream)

        for _ in range(3):
            run()
        _, tmed = time_events(torch, run, reps)
        ttx.ttx_plan_destroy(plan)
        nbytes = n * (c["dtype_a"].itemsize + 2 * c["dtype"].itemsize)
        gbps = nbytes / tmed / 1e9
        out.append(dict(case=c["name"], GBps=round(gbps, 1), pct_of_d2d=round(100 * gbps / d2d, 1),
                        us=round(tmed * 1e6, 1), kernel=kernel))
        del pairs
        torch.cuda.empty_cache()
    g = [o["GBps"] for o in out]
    return dict(cases=out, shapes_tuned_now=tuned, GBps_median=float(np.median(g)), GBps_min=min(g),
                pct_of_d2d_median=round(100 * float(np.median(g)) / d2d, 1))


PACK_CASES = [  # name, dtype code of (A, panels), kind, rows, cols, ld, panel
    ("A_f32_8192x8192_mr16", "F32", "PACK_ROWS", 8192, 8192, 8192, 16),
    ("B_f32_8192x8192_nr16", "F32", "PACK_COLS", 8192, 8192, 8192, 16),
    ("A_f64_6000x5000_mr8_ld6016", "F64", "PACK_ROWS", 6000, 5000, 6016, 8),
    ("B_f64_5000x6000_nr6", "F64", "PACK_COLS", 5000, 6000, 5000, 6),
    ("A_sd_8192x4096_mr16", "F32_F64", "PACK_ROWS", 8192, 4096, 8192, 16),
    ("A_c64_4096x4096_mr4", "C64", "PACK_ROWS", 4096, 4096, 4096, 4),
]


def bench_packing(torch, ttx, d2d, stream, tune_candidates, reps=10):
    """GEMM operand packing (read A, write the panels), one case resident at a
    time, three buffer pairs in rotation as in bench_types."""
    out = []
    tdt = {ttx.F32: torch.float32, ttx.F64: torch.float64, ttx.C32: torch.complex64,
           ttx.C64: torch.complex128}
    for name, code_name, kind_name, rows, cols, ld, panel in PACK_CASES:
        code, kind = getattr(ttx, code_name), getattr(ttx, kind_name)
        ta, tb = ttx.TYPES_OF[code]
        packed, cfgs = ttx.ttx_pack_describe(code, kind, rows, cols, ld, panel)
        ttx.ttx_pack_tune(code, kind, rows, cols, ld, panel, max_candidates=tune_candidates, reps=3)
        real = lambda t: torch.view_as_real(t) if t.is_complex() else t
        pairs = []
        for k in range(3):
            A = torch.empty(ld * cols, dtype=tdt[ta], device="cuda")
            P = torch.empty(packed, dtype=tdt[tb], device="cuda")
            fill_uniform(torch, real(A), 40 + k)
            pairs.append((A, P))
        state = {"i": 0}

        def run():
            state["i"] = (state["i"] + 1) % len(pairs)
            A, P = pairs[state["i"]]
            ttx.ttx_pack(code, kind, rows, cols, ld, panel, 1.0, A.data_ptr(), P.data_ptr(), stream)

        for _ in range(3):
            run()
        _, tmed = time_events(torch, run, reps)
        nbytes = rows * cols * ttx.ELEM_BYTES[ta] + packed * ttx.ELEM_BYTES[tb]
        gbps = nbytes / tmed / 1e9
        out.append(dict(case=name, GBps=round(gbps, 1), pct_of_d2d=round(100 * gbps / d2d, 1),
                        us=round(tmed * 1e6, 1), transpositions=len(cfgs)))
        del pairs
        torch.cuda.empty_cache()
    return out


def bench_contraction(torch, ttx, d2d, stream, reps=10):
    """Transpose-transpose-GEMM-transpose contractions (the workloads'
    CONTRACTIONS), operands resident: the whole ttx_contraction_execute, its
    panel GEMM alone (ttx_gemm_panels on panels of the same extents), the
    rest (transpositions and packing) as the difference, and torch's
    tensordot on the same tensors as a point of comparison."""
    import workloads
    out = []
    for case in workloads.CONTRACTIONS:
        dt = np.dtype(case["dtype"])
        code, tdt = (ttx.F32, torch.float32) if dt == np.float32 else (ttx.F64, torch.float64)
        es = dt.itemsize
        sa, sb, sc = workloads.contraction_sizes(case)
        la, lb, lc = case["labels_a"], case["labels_b"], case["labels_c"]
        plan = ttx.ttx_contraction_create(code, la, sa, lb, sb, lc, sc)
        try:
            info = ttx.ttx_contraction_describe(plan)
            m, n, k, panel = info["m"], info["n"], info["k"], info["panel"]
            T = [torch.empty(int(np.prod(s, dtype=np.int64)), dtype=tdt, device="cuda") for s in (sa, sb, sc)]
            for i, t in enumerate(T):
                fill_uniform(torch, t, 60 + i)
            ws = torch.empty(max(1, info["workspace_bytes"]), dtype=torch.uint8, device="cuda")

            def run():
                ttx.ttx_contraction_execute(plan, case["alpha"], T[0].data_ptr(), T[1].data_ptr(), case["beta"],
                                            T[2].data_ptr(), ws.data_ptr(), stream)

            for _ in range(2):
                run()
            _, t_all = time_events(torch, run, reps)
        finally:
            ttx.ttx_contraction_destroy(plan)
        kb = 64 // panel
        K = -(-k // kb) * kb
        Pa = torch.empty(-(-m // panel) * panel * K, dtype=tdt, device="cuda")
        Pb = torch.empty(-(-n // panel) * panel * K, dtype=tdt, device="cuda")
        fill_uniform(torch, Pa, 70)
        fill_uniform(torch, Pb, 71)
        Cm = torch.empty(m * n, dtype=tdt, device="cuda")

        def gemm():
            ttx.ttx_gemm_panels(code, panel, m, n, k, Pa.data_ptr(), Pb.data_ptr(), Cm.data_ptr(), m, stream)

        gemm()
        _, t_gemm = time_events(torch, gemm, reps)
        del Pa, Pb, Cm
        # torch: column-major tensors are row-major ones with the modes reversed
        ta = T[0].view(*reversed(sa)) if sa else T[0].view(())
        tb = T[1].view(*reversed(sb)) if sb else T[1].view(())
        con = [l for l in la if l in lb]
        dims = ([len(la) - 1 - la.index(l) for l in con], [len(lb) - 1 - lb.index(l) for l in con])
        free = [l for l in reversed(la) if l not in con] + [l for l in reversed(lb) if l not in con]
        want = list(reversed(lc))
        perm = [free.index(l) for l in want]

        def torch_ttgt():
            r = torch.tensordot(ta, tb, dims=dims).permute(*perm)
            return T[2].view(*[case["extent"][l] for l in want]).mul_(case["beta"]).add_(r, alpha=case["alpha"])

        torch_ttgt()
        _, t_torch = time_events(torch, torch_ttgt, reps)
        flops = 2.0 * m * n * k
        rest_bytes = es * ((2 * m * k if info["transposed_a"] else 0) + (2 * k * n if info["transposed_b"] else 0)
                           + m * k + -(-m // panel) * panel * K + k * n + -(-n // panel) * panel * K
                           + m * n * (3 if case["beta"] != 0 else 2))
        t_rest = max(t_all - t_gemm, 1e-9)
        peak = 157.3 if code == ttx.F32 else 78.6
        out.append(dict(case=case["name"], m=m, n=n, k=k, panel=panel, transposed_a=info["transposed_a"],
                        transposed_b=info["transposed_b"], ms=round(t_all * 1e3, 3),
                        TFLOPs=round(flops / t_all / 1e12, 2), gemm_ms=round(t_gemm * 1e3, 3),
                        gemm_TFLOPs=round(flops / t_gemm / 1e12, 2), gemm_frac_of_peak=round(flops / t_gemm / 1e12 / peak, 3),
                        rest_ms=round(t_rest * 1e3, 3), rest_bytes=rest_bytes,
                        rest_GBps=round(rest_bytes / t_rest / 1e9, 1),
                        rest_pct_of_d2d=round(100 * rest_bytes / t_rest / 1e9 / d2d, 1) if d2d else None,
                        torch_tensordot_ms=round(t_torch * 1e3, 3),
                        x_torch=round(t_torch / t_all, 2)))
        log("  %s: %.3f ms (GEMM %.3f ms = %.1f TFLOP/s; rest %.3f ms) vs torch %.3f ms" % (
            case["name"], t_all * 1e3, t_gemm * 1e3, flops / t_gemm / 1e12, t_rest * 1e3, t_torch * 1e3))
        del T, ws
        torch.cuda.empty_cache()
    return out


def side_cases():
    """Shapes timed beside the step: the multiple-leading-dimension and awkward
    shapes (FP64 sub-tensor (384,96,48,32) in outer sizes, (7,1023,33,65) with
    the stride-1 index moved last; both scalar pairs), the literal
    (160,160,160,160) 4D shapes and the literal 24^6 6D shapes."""
    import workloads
    out = []
    for c in workloads.LD_CASES:
        for alpha, beta in workloads.LD_SCALARS:
            out.append(dict(name="%s_a%s_b%s" % (c["name"], alpha, beta), dtype=c["dtype"], size=c["size"],
                            perm=c["perm"], outer_a=c["outer_a"], outer_b=c["outer_b"], alpha=alpha, beta=beta))
    for dtype in (workloads.F32, workloads.F64):
        dn = "f32" if dtype == workloads.F32 else "f64"
        for perm in workloads.LARGE_PERMS["4d"]:
            out.append(dict(name="literal160_%s_p%s" % (dn, "".join(map(str, perm))), dtype=dtype,
                            size=workloads.LITERAL_4D, perm=perm, outer_a=None, outer_b=None, alpha=1.3, beta=0.7))
        for perm in workloads.LARGE_PERMS["6d"]:
            out.append(dict(name="literal24x6_%s_p%s" % (dn, "".join(map(str, perm))), dtype=dtype,
                            size=workloads.LITERAL_6D, perm=perm, outer_a=None, outer_b=None, alpha=1.3, beta=0.7))
    return out


def bench_side(torch, ttx, d2d, stream, tune_candidates, reps=5, tune=True):
    """Each side case through its plan with its size-specialised kernel (tuned
    first when the table has no entry): median of `reps` launches bracketed by
    events.  Shapes under 256 MiB rotate over four buffer sets so that no
    launch finds its own data in the Infinity Cache."""
    import workloads
    out, tuned = [], 0
    for c in side_cases():
        code = ttx.F32 if c["dtype"] == workloads.F32 else ttx.F64
        es = c["dtype"].itemsize
        size_b = [c["size"][p] for p in c["perm"]]
        na = workloads.elements(c["outer_a"] or c["size"])
        nb = workloads.elements(c["outer_b"] or size_b)
        z = c["beta"] == 0
        plan = ttx.ttx_plan_create(code, c["perm"], c["size"], c["outer_a"], c["outer_b"])
        if tune and not ttx.ttx_plan_describe(plan)["config_from_table"][int(z)]:
            log("tuning %s" % c["name"])
            ttx.ttx_tune(code, c["perm"], c["size"], c["outer_a"], c["outer_b"], beta_is_zero=z,
                         max_candidates=tune_candidates, reps=3)
            ttx.ttx_plan_destroy(plan)
            plan = ttx.ttx_plan_create(code, c["perm"], c["size"], c["outer_a"], c["outer_b"])
            tuned += 1
        try:
            ttx.ttx_plan_specialise(plan, z)
        except ttx.TTXError as e:
            log("specialisation failed for %s (%s): generic kernel" % (c["name"], e))
        tdt = torch.float32 if es == 4 else torch.float64
        sets = 4 if (na + nb) * es < (256 << 20) else 1
        bufs = []
        for k in range(sets):
            A = torch.empty(na, dtype=tdt, device="cuda")
            B = torch.empty(nb, dtype=tdt, device="cuda")
            fill_uniform(torch, A, 300 + k)
            fill_uniform(torch, B, 400 + k)
            bufs.append((A, B))
        kernel = ttx.ttx_plan_kernel_name(plan, c["beta"], bufs[0][0].data_ptr(), bufs[0][1].data_ptr())
        state = {"i": 0}

        def run():
            state["i"] = (state["i"] + 1) % len(bufs)
            A, B = bufs[state["i"]]
            ttx.ttx_plan_execute(plan, c["alpha"], A.data_ptr(), c["beta"], B.data_ptr(), stream)

        for _ in range(2):
            run()
        tmin, tmed = time_events(torch, run, reps)
        ttx.ttx_plan_destroy(plan)
        nbytes = workloads.elements(c["size"]) * es * (2 if z else 3)
        gbps = nbytes / tmed / 1e9
        out.append(dict(case=c["name"], GBps=round(gbps, 1), pct_of_d2d=round(100 * gbps / d2d, 1),
                        us=round(tmed * 1e6, 1), bytes=nbytes, kernel=kernel))
        del bufs
        torch.cuda.empty_cache()
    return dict(cases=out, shapes_tuned_now=tuned)


def bench_served(torch, ttx, seconds, rate):
    """Open-loop Poisson trace through the server vs the same trace run one
    synchronised per-call request at a time; a sample of requests is re-run
    alone and compared bitwise with its in-mix result."""
    import workloads
    times, shapes = workloads.served_trace(rate=rate, duration=seconds)
    n = len(times)
    pool_bytes = 2 << 30
    half = pool_bytes // 2
    pool = torch.empty(pool_bytes // 4, dtype=torch.float32, device="cuda")
    fill_uniform(torch, pool, 777)
    base = pool.data_ptr()
    rng = np.random.default_rng(8)
    reqs = ttx._ttx.request_array(n)
    nbytes_total = 0
    max_out = 0
    large_seen = 0
    meta = []
    for i, r in enumerate(shapes):
        es = r["dtype"].itemsize
        ne = workloads.elements(r["size"])
        nb = ne * es
        off_a = int(rng.integers(0, (half - nb) // 256 + 1)) * 256
        off_b = half + int(rng.integers(0, (half - nb) // 256 + 1)) * 256
        k = len(r["perm"])
        row = reqs[i]
        row["dtype"] = ttx.F32 if es == 4 else ttx.F64
        row["n"] = k
        row["perm"][:k] = r["perm"]
        row["size"][:k] = r["size"]
        row["alpha"] = r["alpha"]
        row["beta"] = r["beta"]
        row["A"] = base + off_a
        row["B_in"] = base + off_b
        keep = i % 997 == 0 or (r["large"] and large_seen < 64)
        large_seen += 1 if r["large"] else 0
        row["keep_result"] = 1 if keep else 0
        nbytes_total += nb * (2 if r["beta"] == 0 else 3)
        max_out = max(max_out, nb)
        meta.append((r, off_a, off_b, nb))
    offsets = (np.asarray(times) * 1e9).astype(np.int64)
    torch.cuda.synchronize()
    log("serving %d requests over %.1f s" % (n, seconds))
    s = ttx.ttx_server_create(slots=SLOTS, arena_bytes=16 << 30)
    try:
        tickets = ttx.ttx_server_replay_clients(s, reqs, offsets, CLIENTS)
        ttx.ttx_server_drain(s)
        st = ttx.ttx_server_get_stats(s)
        # the mix check: each kept result against the same request alone
        hip = hip_runtime()
        scratch = torch.empty(max_out + 256, dtype=torch.uint8, device="cuda")
        served = torch.empty_like(scratch)
        stream = torch.cuda.current_stream().cuda_stream
        checked = mismatched = 0
        for i in range(n):
            if not reqs[i]["keep_result"] or tickets[i] == 0:
                continue
            r, off_a, off_b, nb = meta[i]
            ptr, _ = ttx.ttx_server_result(s, int(tickets[i]))
            torch.cuda.synchronize()
            assert hip.hipMemcpy(served.data_ptr(), ptr, nb, 3) == 0
            plan = ttx.ttx_plan_create(ttx.F32 if r["dtype"].itemsize == 4 else ttx.F64, r["perm"], r["size"])
            ttx.ttx_plan_execute_split(plan, r["alpha"], base + off_a, r["beta"], base + off_b,
                                       scratch.data_ptr(), stream)
            ttx.ttx_plan_destroy(plan)
            torch.cuda.synchronize()
            checked += 1
            mismatched += 0 if torch.equal(scratch[:nb], served[:nb]) else 1
            ttx.ttx_server_release(s, int(tickets[i]))
    finally:
        ttx.ttx_server_destroy(s)
    log("sequential per-call baseline")
    scratch = torch.empty(max_out + 256, dtype=torch.uint8, device="cuda")
    lat = ttx.ttx_replay_sequential(reqs, offsets, scratch.data_ptr(), scratch.numel(),
                                    torch.cuda.current_stream().cuda_stream)
    span = float(np.max(times + lat * 1e-6) - times[0])
    saturated = bench_saturated(torch, ttx, reqs, meta, scratch)
    del pool, scratch
    return dict(requests=n, rate_per_s=rate, seconds=seconds, algorithmic_bytes=nbytes_total, clients=CLIENTS,
                served=dict(GBps=round(st["throughput_gbps"], 1), p50_us=round(st["p50_us"], 1),
                            p99_us=round(st["p99_us"], 1), max_us=round(st["max_us"], 1),
                            batches=st["batches"], mean_batch=round(st["mean_batch"], 2),
                            rejected=st["rejected"], budget_GB=round(st["budget_bytes"] / 1e9, 1),
                            peak_in_use_GB=round(st["peak_in_use_bytes"] / 1e9, 3), slots=SLOTS),
                sequential=dict(GBps=round(nbytes_total / span / 1e9, 1), p50_us=round(_pct(lat, 50), 1),
                                p99_us=round(_pct(lat, 99), 1), max_us=round(float(np.max(lat)), 1)),
                throughput_ratio=round(st["throughput_gbps"] / (nbytes_total / span / 1e9), 2),
                mix_check=dict(compared=checked, bitwise_mismatches=mismatched),
                saturated=saturated)


def bench_saturated(torch, ttx, reqs, meta, scratch, budget_bytes=8e9):
    """Capacity: the trace's first requests (up to ~8 GB of algorithmic
    traffic) all arrive at once, through the server and through the
    sequential per-call loop; throughput = bytes / (last completion - arrival)."""
    nb = np.array([m[3] * (2 if m[0]["beta"] == 0 else 3) for m in meta], dtype=np.float64)
    m = int(np.searchsorted(np.cumsum(nb), budget_bytes)) + 1
    m = max(1, min(m, len(meta)))
    sub = ttx._ttx.request_array(m)     # zeroed, so the unnamed outer-size fields stay zero
    for f in reqs.dtype.names:
        sub[f] = reqs[f][:m]
    sub["keep_result"] = 0
    zeros = np.zeros(m, dtype=np.int64)
    total = float(nb[:m].sum())
    log("saturated: %d requests at once (%.2f GB)" % (m, total / 1e9))
    s = ttx.ttx_server_create(slots=SLOTS, arena_bytes=16 << 30)
    try:
        ttx.ttx_server_replay_clients(s, sub, zeros, CLIENTS)
        ttx.ttx_server_drain(s)
        st = ttx.ttx_server_get_stats(s)
    finally:
        ttx.ttx_server_destroy(s)
    lat = ttx.ttx_replay_sequential(sub, zeros, scratch.data_ptr(), scratch.numel(),
                                    torch.cuda.current_stream().cuda_stream)
    seq_span = float(np.max(lat)) * 1e-6
    return dict(requests=m, algorithmic_bytes=int(total), clients=CLIENTS, slots=SLOTS,
                served=dict(GBps=round(st["throughput_gbps"], 1), p50_us=round(st["p50_us"], 1),
                            p99_us=round(st["p99_us"], 1), batches=st["batches"],
                            mean_batch=round(st["mean_batch"], 2)),
                sequential=dict(GBps=round(total / seq_span / 1e9, 1), p50_us=round(_pct(lat, 50), 1),
                                p99_us=round(_pct(lat, 99), 1)),
                throughput_ratio=round(st["throughput_gbps"] / (total / seq_span / 1e9), 2))


def compact_line(full, detail_path=None):
    """The one JSON line bench.py prints: the headline, the roofline and CPU
    baseline, and one-number summaries of the side measurements; the per-case
    detail goes to the side file (``detail_path``)."""
    def pick(d, *keys):
        return {k: d[k] for k in keys if d is not None and k in d} if d else None

    line = pick(full, "metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
                "scaling", "vs_baseline", "dtype", "data", "pct_of_d2d")
    cfg = full["config"]
    line["config"] = dict(workload=cfg["workload"], cases=cfg["cases"], bytes_per_step=cfg["bytes_per_step"],
                          entry_point="ttx_plan_execute + ttx_plan_specialise"
                          if "specialise" in cfg["entry_point"] else "ttx_transpose (generic kernels)",
                          parallelism=cfg["parallelism"])
    c = full.get("ceilings") or {}
    line["ceilings_GBps"] = {k: v["GBps"] for k, v in c.items()}
    line["per_perm_GBps"] = full.get("per_perm_GBps")
    v = full.get("verification")
    line["verified"] = None if v is None else v["verified"]
    if v is not None:
        line["verification"] = pick(v, "elements_compared", "differing_elements", "max_ulp")
    line["roofline"] = pick(full["roofline"], "bound", "achieved", "peak", "unit", "frac", "traffic", "kernel",
                            "avg_launch_us", "algorithmic_bytes_per_launch", "launches")
    cpu = full.get("cpu_baseline")
    if cpu:
        host = cpu.get("host") or {}
        line["cpu_baseline"] = dict(pick(cpu, "value", "unit", "cores", "kind", "sample"),
                                    one_thread_GBps=(cpu.get("one_thread") or {}).get("value"),
                                    host_cpus=host.get("usable_cpus"), host_model=host.get("model"))
    else:
        line["cpu_baseline"] = None
    g = full.get("per_call_generic")
    line["per_call_generic_GBps"] = g["value"] if g else None
    b = full.get("batched")
    if b:
        line["batched"] = dict(GBps=b["batched"]["GBps"], per_call_GBps=b["per_call"]["GBps"],
                               x_per_call=b["speedup"], p50_ms=b["batched"]["makespan_p50_ms"],
                               p99_ms=b["batched"]["makespan_p99_ms"], target_x=3.0)
    sv = full.get("served")
    if sv:
        sat = sv.get("saturated") or {}
        line["served"] = dict(GBps=sv["served"]["GBps"], seq_GBps=sv["sequential"]["GBps"],
                              x_seq=sv["throughput_ratio"], p50_us=sv["served"]["p50_us"],
                              p99_us=sv["served"]["p99_us"], seq_p50_us=sv["sequential"]["p50_us"],
                              seq_p99_us=sv["sequential"]["p99_us"],
                              saturated_x_seq=sat.get("throughput_ratio"),
                              mix_mismatches=sv["mix_check"]["bitwise_mismatches"], target_x=3.0)
    sd = full.get("side")
    if sd:
        line["side_pct_of_d2d"] = {k: min(o["pct_of_d2d"] for o in sd["cases"] if o["case"].startswith(k))
                                   for k in ("ld_f64", "awkward", "literal160", "literal24x6")
                                   if any(o["case"].startswith(k) for o in sd["cases"])}
    ot = full.get("other_types")
    if ot:
        pcts = {o["case"]: o["pct_of_d2d"] for o in ot["cases"]}
        line["other_types_pct_of_d2d"] = dict(median=ot["pct_of_d2d_median"], min=min(pcts.values()),
                                              weakest=min(pcts, key=pcts.get))
    pk = full.get("packing")
    if pk:
        line["packing_pct_of_d2d_min"] = min(o["pct_of_d2d"] for o in pk)
    ct = full.get("contraction")
    if ct:
        line["contraction"] = {o["case"]: dict(ms=o["ms"], TFLOPs=o["TFLOPs"], gemm_frac_of_peak=o["gemm_frac_of_peak"],
                                               x_torch=o["x_torch"]) for o in ct}
    sp = full.get("specialised")
    if sp:
        line["specialised_vs_generic_step"] = round(sp["step_GBps_specialised"] / sp["step_GBps_generic"], 3)
    line["detail"] = detail_path
    return line


# ---------------------------------------------------------------------------------------
def main():
    args = parse_args()
    if args.traffic_from:
        traffic_from(*args.traffic_from, out_path=args.traffic_out)
        return 0
    if args.summarize_counters:
        summarize_counters(args.summarize_counters)
        return
    if args.summarize_trace:
        summarize_trace(args.summarize_trace)
        return 0
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        return 2
    if args.profile_run:
        args.steps, args.warmup, args.no_cpu_baseline = 2, 1, True
        args.no_batched = args.no_served = args.no_side = True

    import torch
    import paper_1607_01249_amd as ttx

    ttx.lib()   # raises when the HIP library is not built
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream().cuda_stream
    if args.profile_batched:
        # the 1 GiB copy kernel first: the counter runs calibrate against it
        src = torch.empty((1 << 30) // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        fill_uniform(torch, src, 1)
        for _ in range(3):
            ttx.ttx_copy_kernel(src.data_ptr(), dst.data_ptr(), 1 << 30, stream)
        torch.cuda.synchronize()
        del src, dst
        print(json.dumps(bench_batched(torch, ttx, reps=5, tune=False)))
        return 0
    if args.only_contraction:
        print(json.dumps(bench_contraction(torch, ttx, None, stream, reps=5)))
        return 0
    cases = make_cases(args.literal)
    log("allocating %d cases (%.1f GiB)" % (len(cases), sum(2 * c["elements"] * c["dtype"].itemsize for c in cases) / 2 ** 30))
    for i, c in enumerate(cases):
        tdt = torch.float32 if c["dtype"].itemsize == 4 else torch.float64
        c["A"] = torch.empty(c["elements"], dtype=tdt, device="cuda")
        c["B"] = torch.empty(c["elements"], dtype=tdt, device="cuda")
        fill_uniform(torch, c["A"], c["seed_a"])
        fill_uniform(torch, c["B"], c["seed_b"])
        c["code"] = ttx.F32 if tdt == torch.float32 else ttx.F64
    torch.cuda.synchronize()

    # Solution lookup before search (Sec. 2.1): shipped table first, tune the rest.
    if os.path.exists(TABLE) and not args.retune:
        ttx.ttx_tune_table_load(TABLE)
    tune_t0 = time.time()
    tuned = 0
    for c in cases:
        plan = ttx.ttx_plan_create(c["code"], c["perm"], c["size"])
        info = ttx.ttx_plan_describe(plan)
        ttx.ttx_plan_destroy(plan)
        z = 1 if c["beta"] == 0 else 0
        if not info["config_from_table"][z]:
            if args.profile_run:
                raise SystemExit("--profile-run needs every case in the tune table (%s)" % c["name"])
            log("tuning %s" % c["name"])
            ttx.ttx_tune(c["code"], c["perm"], c["size"], beta_is_zero=bool(z),
                         max_candidates=args.tune_candidates, reps=3)
            tuned += 1
    tune_s = time.time() - tune_t0
    if args.save_table:
        ttx.ttx_tune_table_save(args.save_table)
    # The step runs each case's plan with its size-specialised kernel (Sec. 2.1:
    # a solution per transposition, sizes as constants), compiled here, before
    # the timed region; a case whose compilation fails keeps its generic kernel.
    spec_t0 = time.time()
    n_spec = 0
    for c in cases:
        c["plan"] = ttx.ttx_plan_create(c["code"], c["perm"], c["size"])
        if not args.generic:
            try:
                n_spec += ttx.ttx_plan_specialise(c["plan"], c["beta"] == 0)
            except ttx.TTXError as e:
                log("specialisation failed for %s (%s): generic kernel" % (c["name"], e))
        c["kernel"] = ttx.ttx_plan_kernel_name(c["plan"], c["beta"], c["A"].data_ptr(), c["B"].data_ptr())
        c["config"] = ttx.ttx_plan_describe(c["plan"])["config"][1 if c["beta"] == 0 else 0]
    spec_s = time.time() - spec_t0

    log("measuring ceilings")
    ceil = measure_ceilings(torch, ttx)
    d2d = ceil["hipMemcpy_d2d"]["GBps"]

    def step(events=None, generic=args.generic):
        for i, c in enumerate(cases):
            if events is not None:
                events[i].record()
            if generic:
                ttx.ttx_transpose(c["code"], len(c["perm"]), c["perm"], c["size"], None, None,
                                  c["alpha"], c["A"].data_ptr(), c["beta"], c["B"].data_ptr(), stream)
            else:
                ttx.ttx_plan_execute(c["plan"], c["alpha"], c["A"].data_ptr(), c["beta"], c["B"].data_ptr(), stream)
        if events is not None:
            events[len(cases)].record()

    log("warm-up")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    events = [[torch.cuda.Event(enable_timing=True) for _ in range(len(cases) + 1)]
              for _ in range(args.steps)]
    log("timing %d steps" % args.steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(events[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    step_bytes = sum(c["bytes"] for c in cases)
    value = step_bytes * args.steps / wall / 1e9
    per_call_generic = None
    if not args.generic and not args.profile_run:
        # the same step through the per-call entry point with the generic kernels
        step(generic=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step(generic=True)
        torch.cuda.synchronize()
        v = step_bytes * args.steps / (time.perf_counter() - t0) / 1e9
        per_call_generic = dict(value=round(v, 1), pct_of_d2d=round(100 * v / d2d, 1), entry_point="ttx_transpose")
    per_case, by_kernel = [], {}
    for i, c in enumerate(cases):
        durs = [events[k][i].elapsed_time(events[k][i + 1]) * 1e-3 for k in range(args.steps)]
        med = float(np.median(durs))
        gbps = c["bytes"] / med / 1e9
        per_case.append(dict(case=c["name"], perm=list(c["perm"]), size=list(c["size"]),
                             dtype="f32" if c["dtype"].itemsize == 4 else "f64", beta=c["beta"],
                             GBps=round(gbps, 1), pct_of_d2d=round(100 * gbps / d2d, 1),
                             us=round(med * 1e6, 1), kernel=c["kernel"]))
        k = by_kernel.setdefault(c["kernel"], dict(time=0.0, bytes=0, launches=0))
        k["time"] += sum(durs)
        k["bytes"] += c["bytes"] * args.steps
        k["launches"] += args.steps
    dom_name, dom = max(by_kernel.items(), key=lambda kv: kv[1]["time"])
    achieved = dom["bytes"] / dom["time"] / 1e9
    bytes_per_launch = dom["bytes"] / dom["launches"]
    traffic = None   # counter bytes per launch, only while the kernel sources are unchanged
    if os.path.exists(TRAFFIC):
        with open(TRAFFIC) as f:
            tr = json.load(f)
        if tr.get("source_hash") == kernel_source_hash() and dom_name in tr.get("kernels", {}):
            traffic = tr["kernels"][dom_name]["traffic_bytes"]
    roofline = dict(bound="hbm", achieved=round(achieved, 1), peak=PEAK_HBM_GBPS, unit="GB/s",
                    frac=round(achieved / PEAK_HBM_GBPS, 4), traffic=traffic,
                    kernel=dom_name, launches=dom["launches"],
                    avg_launch_us=round(dom["time"] / dom["launches"] * 1e6, 2),
                    algorithmic_bytes_per_launch=int(bytes_per_launch))
    if args.dominant_out and not args.profile_run:
        with open(args.dominant_out, "w") as f:
            json.dump(dict(kernel=dom_name, bytes_per_launch=bytes_per_launch,
                           avg_launch_us=roofline["avg_launch_us"]), f)

    # The CPU-baseline leg: the oracle timed on the host, and every case's GPU
    # output compared with it (outside the timed region).
    cpu = verification = None
    if not args.no_cpu_baseline:
        log("CPU oracle baseline and verification")
        cpu, verification = cpu_baseline(torch, ttx, cases, stream)

    specialised = None
    if not args.no_specialised and not args.profile_run:
        log("size-specialised kernels")
        specialised = bench_specialised(torch, ttx, cases, d2d, stream)

    for c in cases:   # the large cases' buffers and plans are not needed any more
        c.pop("A", None)
        c.pop("B", None)
        ttx.ttx_plan_destroy(c.pop("plan"))
    torch.cuda.empty_cache()
    side = None
    if not args.no_side and not args.profile_run:
        log("side shapes: leading dimensions, awkward extents, literal 160^4 and 24^6")
        side = bench_side(torch, ttx, d2d, stream, args.tune_candidates)
    batched = None
    if not args.no_batched:
        log("batched: 512 problems")
        batched = bench_batched(torch, ttx)
    served = None
    if not args.no_served:
        served = bench_served(torch, ttx, args.serve_seconds, args.serve_rate)

    cplx = packing = None
    if not args.no_types and not args.profile_run:
        log("complex and mixed-precision cases")
        cplx = bench_types(torch, ttx, d2d, stream, args.tune_candidates, specialise=not args.generic)
        log("GEMM operand packing")
        packing = bench_packing(torch, ttx, d2d, stream, args.tune_candidates)
    contraction = None
    if not args.no_contraction and not args.profile_run:
        log("tensor contractions (transpose-transpose-GEMM-transpose)")
        contraction = bench_contraction(torch, ttx, d2d, stream)
    if args.save_table:
        ttx.ttx_tune_table_save(args.save_table)

    gbps_cases = [p["GBps"] for p in per_case]
    weakest = min(per_case, key=lambda p: p["GBps"])
    full = dict(
        metric=METRIC, value=round(value, 1), unit="GB/s", n_gpus=1, steps=args.steps,
        warmup=args.warmup, ms_per_step=round(wall / args.steps * 1e3, 3), higher_is_better=True,
        scaling="weak", vs_baseline=None, dtype="f32+f64", data="synthetic",
        config=dict(workload="paper-shaped transpositions, ~200 MiB per tensor: 4D/5D/6D x FP32/FP64 x "
                             "(beta=0.7, beta=0), alpha=1.3, %d cases per step%s" %
                             (len(cases), " + literal 160^4" if args.literal else ""),
                    cases=len(cases), bytes_per_step=step_bytes, layout="column-major",
                    entry_point="ttx_transpose (per call, generic kernels)" if args.generic else
                    "ttx_plan_execute, one plan per case with its size-specialised kernel (ttx_plan_specialise, "
                    "%d of %d compiled in %.1f s before timing)" % (n_spec, len(cases), spec_s),
                    parallelism="single GPU"),
        per_call_generic=per_call_generic,
        pct_of_d2d=round(100 * value / d2d, 1),
        ceilings=ceil,
        per_perm_GBps=dict(min=min(gbps_cases), median=float(np.median(gbps_cases)), max=max(gbps_cases),
                           weakest=weakest["case"], weakest_pct_of_d2d=weakest["pct_of_d2d"]),
        verification=verification,
        roofline=roofline, cpu_baseline=cpu, specialised=specialised, side=side, batched=batched, served=served,
        other_types=cplx,
        packing=packing,
        contraction=contraction,
        tuning=dict(table=os.path.relpath(TABLE, ROOT) if os.path.exists(TABLE) else None,
                    shapes_tuned_now=tuned, seconds=round(tune_s, 1)),
        per_perm=per_case,
    )
    line = compact_line(full, args.detail_out)
    if args.detail_out:
        d = os.path.dirname(os.path.abspath(args.detail_out))
        os.makedirs(d, exist_ok=True)
        with open(args.detail_out, "w") as f:
            json.dump(full, f, indent=1)
    print(json.dumps(line, separators=(",", ":")), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
