"""Host-side sweep (no GPU): every shape of the batched workload and of the
first part of the served trace is planned, described, and given its kernel
name and batched descriptor, for both data types and aligned and misaligned
pointers.  Catches planner defects on the long tail of random shapes."""
import paper_1607_01249_amd as ttx
import workloads


def _shapes():
    probs = workloads.batched_problems()
    _, served = workloads.served_trace(duration=1.5)
    return [(p["perm"], p["size"]) for p in probs] + [(r["perm"], r["size"]) for r in served]


def test_plan_every_workload_shape():
    shapes = _shapes()
    assert len(shapes) > 20000
    base = 1 << 40
    for i, (perm, size) in enumerate(shapes):
        dt = ttx.F32 if i % 3 else ttx.F64
        p = ttx.ttx_plan_create(dt, perm, size)
        try:
            d = ttx.ttx_plan_describe(p)
            for beta in (0.0, 0.5):
                name = ttx.ttx_plan_kernel_name(p, beta, base, base + (1 << 36))
                assert name.startswith("k_"), name
                name = ttx.ttx_plan_kernel_name(p, beta, base + 4 * (i % 2), base + (1 << 36) + 8)
                assert name.startswith("k_"), name
            # the config the planner picked is one it accepts back
            cfg = d["config_raw"][0]
            ttx.ttx_plan_set_config(p, 0, cfg)
        finally:
            ttx.ttx_plan_destroy(p)


def test_batch_plan_every_served_shape():
    _, served = workloads.served_trace(duration=0.5)
    base = 1 << 40
    qs = []
    for r in served:
        nbytes = workloads.elements(r["size"]) * r["dtype"].itemsize
        A = base
        base += nbytes + 256
        qs.append(ttx.make_problem(ttx.F32 if r["dtype"].itemsize == 4 else ttx.F64, r["perm"], r["size"],
                                   r["alpha"], A, r["beta"], base))
        base += nbytes + 256
    cfgs, tiles = ttx.ttx_batch_plan(qs)
    assert len(cfgs) == len(qs) and min(tiles) >= 1
