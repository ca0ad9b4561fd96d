"""Refines a tune table's entries for size-specialised execution with the
workgroup dimensions (threads per workgroup, LDS row padding, line-aligned
A runs).

For each problem given, the plan's configuration for specialised execution
(the table's `j:` entry, else its generic entry) is the base; every workgroup
variant of it (ttx_tune_variants) is compiled as a size-specialised kernel
and timed the way a throughput loop runs it: back-to-back launches that
rotate over three buffer pairs (so that each launch finds the data of the
two before it in the 256 MiB Infinity Cache, not its own), median of the
launch times, in several rounds with the base re-timed in each.  A variant replaces the base only when its median is lower by at
least `--margin` in every round.  The result is written as `j:` entries of
a new table file (the generic entries are copied unchanged).

    python paper_1607_01249_amd/tune/refine_workgroups.py IN OUT [--cases large|complex|mixed|all]
           [--only NAME ...] [--shapes] [--large-only] [--pipelined-only]

Needs a GPU.  Blocks for a few seconds per problem.
"""
import argparse
import os
import statistics
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def table_key(info, z):
    """The tune table key of a plan (the format ttx writes: dtype, beta == 0, merged problem)."""
    j = lambda xs: ",".join(map(str, xs))
    return "d%d:b%d:n%d:s%s:p%s:a%s:o%s" % (info["dtype"], z, info["n"], j(info["size"]), j(info["perm"]),
                                          j(info["stride_a"]), j(info["stride_b"]))


def config_text(c):
    """A config as a table line's middle field."""
    f = [c.family, c.tile_a, c.tile_b, c.threads, c.flags, c.group_a, c.group_b, c.n_order]
    f += list(c.order[:c.n_order])
    s = " ".join(map(str, f))
    if c.tile_c > 1:
        s += " c%d" % c.tile_c
    if c.lds_pad != 1:
        s += " l%d" % c.lds_pad
    return s


def _timed(ttx, torch, plan, case, pairs, stream, launches=13):
    """Median launch time (us), launches rotating over the (A, B) pointer pairs."""
    for k in range(3):
        A, B = pairs[k % len(pairs)]
        ttx.ttx_plan_execute_c(plan, case["alpha"], A, case["beta"], B, B, stream)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(launches + 1)]
    for r in range(launches):
        A, B = pairs[r % len(pairs)]
        ev[r].record()
        ttx.ttx_plan_execute_c(plan, case["alpha"], A, case["beta"], B, B, stream)
    ev[launches].record()
    torch.cuda.synchronize()
    return statistics.median(ev[r].elapsed_time(ev[r + 1]) * 1e3 for r in range(launches))


def large_variants(ttx, code, perm, size, base):
    """The base with each run-time-only large moved tile instead of its own,
    at 256 and 512 threads, line-aligned A runs on and off (moved bases only)."""
    if base.family != ttx.FAMILY_MOVED or base.flags & ttx.CFG_DENSE:
        return []
    out = []
    for ta, tb in ttx.ttx_tile_shapes(code, ttx.FAMILY_MOVED, run_time_only=True):
        for threads in (256, 512):
            for align in (0, ttx.CFG_ALIGN_A):
                v = ttx.Config.from_buffer_copy(base)
                v.tile_a, v.tile_b, v.threads, v.lds_pad = ta, tb, threads, 1
                v.flags = (v.flags & ~ttx.CFG_ALIGN_A) | align
                out.append(v)
    return out


def pipelined_variants(ttx, code, perm, size, base):
    """The base as a pipelined persistent grid (TTX_CFG_PIPELINED), at its
    own workgroup size and at the other of 256 and 512 threads (moved and
    preserved bases, not dense ones)."""
    if base.family not in (ttx.FAMILY_MOVED, ttx.FAMILY_PRESERVED) or base.flags & ttx.CFG_DENSE:
        return []
    out = []
    for threads in sorted({base.threads, 512 if base.threads == 256 else 256}):
        v = ttx.Config.from_buffer_copy(base)
        v.flags |= ttx.CFG_PIPELINED
        v.threads = threads
        out.append(v)
    return out


def shape_variants(ttx, code, perm, size, base):
    """Moved-family configs with the base's index groups, loop order and
    flags and every other tile shape of the menu that fits this layout (and
    every run-time-only large tile),
    each at 256 and 512 threads per workgroup, with line-aligned A runs on
    and off where they apply (the first search stage ranks shapes at 256
    threads only)."""
    if base.family != ttx.FAMILY_MOVED or base.flags & ttx.CFG_DENSE:
        return []
    cands, _ = ttx.ttx_tune_candidates(code, perm, size, max_candidates=-1, cap=200000)
    shapes = {(c.tile_a, c.tile_b) for c in cands
              if c.family == ttx.FAMILY_MOVED and not c.flags & ttx.CFG_DENSE and
              (c.group_a, c.group_b) == (base.group_a, base.group_b)}
    # and the larger tiles that exist only as run-time compiled kernels
    shapes = sorted(shapes | set(ttx.ttx_tile_shapes(code, ttx.FAMILY_MOVED, run_time_only=True)))
    out = []
    for ta, tb in shapes:
        for threads in (256, 512):
            for align in (0, ttx.CFG_ALIGN_A):
                v = ttx.Config.from_buffer_copy(base)
                v.tile_a, v.tile_b, v.threads, v.lds_pad = ta, tb, threads, 1
                v.flags = (v.flags & ~ttx.CFG_ALIGN_A) | align
                if (ta, tb, threads, v.flags) != (base.tile_a, base.tile_b, base.threads, base.flags):
                    out.append(v)
    return out


def refine(cases, rounds=2, margin=0.02, log=print, shapes=False, large_only=False, pipelined_only=False):
    """{key: (config, usec)} of the variants that beat their base (with
    shapes, also the other menu tile shapes of moved-family bases; with
    large_only, the base against its large run-time-only tiles alone; with
    pipelined_only, against its pipelined persistent grids alone)."""
    import torch
    import paper_1607_01249_amd as ttx
    stream = ttx.current_stream()
    out = {}
    for case in cases:
        code, perm, size = case["code"], case["perm"], case["size"]
        z = 1 if case["beta"] == 0 else 0
        plan = ttx.ttx_plan_create(code, perm, size)
        try:
            ttx.ttx_plan_specialise(plan, z)
            info = ttx.ttx_plan_describe(plan)
            base = ttx.Config.from_buffer_copy(info["config_raw"][z])
        finally:
            ttx.ttx_plan_destroy(plan)
        if info["family"] not in ("moved", "preserved"):
            continue
        if large_only:
            variants = [base] + large_variants(ttx, code, perm, size, base)
        elif pipelined_only:
            variants = [base] + pipelined_variants(ttx, code, perm, size, base)
        else:
            variants = ttx.ttx_tune_variants(code, perm, size, base)
            if shapes:
                variants += shape_variants(ttx, code, perm, size, base)
        bufs = [(torch.empty(max(1, info["extent_a_bytes"] // 4 + 4), dtype=torch.float32, device="cuda").uniform_(-1, 1),
                 torch.empty(max(1, info["extent_b_bytes"] // 4 + 4), dtype=torch.float32, device="cuda").uniform_(-1, 1))
                for _ in range(3)]
        pairs = [(a.data_ptr(), b.data_ptr()) for a, b in bufs]
        plans, kept_v = [], []
        for v in variants:
            p = ttx.ttx_plan_create(code, perm, size)
            try:
                ttx.ttx_plan_set_config(p, z, v)
            except ttx.TTXError:   # a shape whose tile does not fit this workgroup
                ttx.ttx_plan_destroy(p)
                continue
            ttx.ttx_plan_specialise(p, z)
            plans.append(p)
            kept_v.append(v)
        variants = kept_v
        times = [[] for _ in variants]
        for _ in range(rounds):
            for i, p in enumerate(plans):
                times[i].append(_timed(ttx, torch, p, case, pairs, stream))
        for p in plans:
            ttx.ttx_plan_destroy(p)
        best = min(range(len(variants)), key=lambda i: max(times[i]))
        gain = [1 - times[best][r] / times[0][r] for r in range(rounds)]
        kept = best != 0 and min(gain) >= margin
        al = lambda c: ("a" if c.flags & ttx.CFG_ALIGN_A else "") + ("P" if c.flags & ttx.CFG_PIPELINED else "")
        other = min(range(1, len(variants)), key=lambda i: max(times[i])) if len(variants) > 1 else 0
        log("%s: base %dx%d t%d p%d%s %.1f us, best %dx%d t%d p%d%s %.1f us (%+.1f%%)%s; best other %dx%d t%d p%d%s "
            "%.1f us" % (
                case["name"], base.tile_a, base.tile_b, base.threads, base.lds_pad, al(base), max(times[0]),
                variants[best].tile_a, variants[best].tile_b, variants[best].threads, variants[best].lds_pad,
                al(variants[best]), max(times[best]), -100 * min(gain), " -> kept" if kept else "",
                variants[other].tile_a, variants[other].tile_b, variants[other].threads, variants[other].lds_pad,
                al(variants[other]), max(times[other])))
        if kept:
            out[table_key(info, z)] = (variants[best], max(times[best]))
        del bufs
        torch.cuda.empty_cache()
    return out


def write_table(src, dst, entries):
    """Copies src to dst with `j:` entries for `entries` (replacing any there)."""
    lines = open(src).read().splitlines()
    keep = [l for l in lines if not any(l.startswith("j:" + k + " |") for k in entries)]
    for k, (c, us) in sorted(entries.items()):
        keep.append("j:%s | %s | %.3f" % (k, config_text(c), us))
    with open(dst, "w") as f:
        f.write("\n".join(keep) + "\n")


def bench_cases(which):
    """The throughput problems, as dicts with code, perm, size, alpha, beta (complex scalars)."""
    import paper_1607_01249_amd as ttx
    import workloads
    import numpy as np
    tcode = {np.dtype(np.float32): ttx.F32, np.dtype(np.float64): ttx.F64,
             np.dtype(np.complex64): ttx.C32, np.dtype(np.complex128): ttx.C64}
    out = []
    if which in ("large", "all"):
        for c in workloads.large_cases():
            out.append(dict(name=c["name"], code=tcode[np.dtype(c["dtype"])], perm=c["perm"], size=c["size"],
                            alpha=complex(c["alpha"]), beta=complex(c["beta"])))
    for kind, gen in (("complex", workloads.complex_cases), ("mixed", workloads.mixed_cases)):
        if which in (kind, "all"):
            for c in gen():
                code = ttx.CODE_OF[(tcode[np.dtype(c["dtype_a"])], tcode[np.dtype(c["dtype"])])]
                out.append(dict(name=c["name"], code=code, perm=c["perm"], size=c["size"],
                                alpha=complex(c["alpha"]), beta=complex(c["beta"])))
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("table_in")
    ap.add_argument("table_out")
    ap.add_argument("--cases", default="large", choices=["large", "complex", "mixed", "all"])
    ap.add_argument("--only", nargs="*", default=None, help="case names")
    ap.add_argument("--rounds", type=int, default=2)
    ap.add_argument("--margin", type=float, default=0.02)
    ap.add_argument("--shapes", action="store_true",
                    help="also try the other menu tile shapes of moved-family bases (256/512 threads, "
                         "line-aligned A runs on and off)")
    ap.add_argument("--large-only", action="store_true",
                    help="time each base against its run-time-only large moved tiles only")
    ap.add_argument("--pipelined-only", action="store_true",
                    help="time each base against its pipelined persistent grids (TTX_CFG_PIPELINED) only")
    args = ap.parse_args()
    import paper_1607_01249_amd as ttx
    ttx.ttx_tune_table_clear()
    ttx.ttx_tune_table_load(args.table_in)
    cases = bench_cases(args.cases)
    if args.only:
        cases = [c for c in cases if c["name"] in args.only]
    entries = refine(cases, args.rounds, args.margin, log=lambda m: print(m, flush=True), shapes=args.shapes,
                     large_only=args.large_only, pipelined_only=args.pipelined_only)
    write_table(args.table_in, args.table_out, entries)
    print("%d of %d entries refined -> %s" % (len(entries), len(cases), args.table_out), flush=True)


if __name__ == "__main__":
    main()
