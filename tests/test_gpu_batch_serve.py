"""GPU parity of batched execution and serving.

Batched: the 512-problem workload (N in 2..6, random permutations, element
counts log-uniform in 4K..4M, 70% FP32, alpha and beta uniform in [-2, 2],
beta = 0 for a quarter) run as one persistent graph-captured launch must
match the oracle problem by problem and be bitwise equal to the per-call
path; graph replays repeat the eager result.

Served: requests replayed through the server give the same bits as the same
request run alone through ttx_transpose, and as the oracle.
"""
import sys

import numpy as np
import pytest

import oracle
import paper_1607_01249_amd as ttx
import workloads
from gpu_util import F32, assert_parity

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _tdt(dtype):
    import torch
    return torch.float32 if np.dtype(dtype) == F32 else torch.float64


class Batch:
    """Host and device copies of a list of workload problems."""

    def __init__(self, probs, seed=100):
        import torch
        self.probs = probs
        self.A, self.B0, self.dA, self.dB = [], [], [], []
        for i, p in enumerate(probs):
            n = workloads.elements(p["size"])
            a = workloads.uniform(n, p["dtype"], seed + 2 * i)
            b = workloads.uniform(n, p["dtype"], seed + 2 * i + 1)
            self.A.append(a)
            self.B0.append(b)
            self.dA.append(torch.from_numpy(a).cuda())
            self.dB.append(torch.from_numpy(b).cuda())
        torch.cuda.synchronize()

    def reset_b(self):
        import torch
        for d, b in zip(self.dB, self.B0):
            d.copy_(torch.from_numpy(b))
        torch.cuda.synchronize()

    def problems(self):
        return [ttx.make_problem(ttx.F32 if p["dtype"].itemsize == 4 else ttx.F64, p["perm"],
                                 p["size"], p["alpha"], a.data_ptr(), p["beta"], b.data_ptr())
                for p, a, b in zip(self.probs, self.dA, self.dB)]

    def results(self):
        import torch
        torch.cuda.synchronize()
        return [d.cpu().numpy() for d in self.dB]

    def oracle(self):
        out = []
        for p, a, b in zip(self.probs, self.A, self.B0):
            r = b.copy()
            assert oracle.transpose(p["perm"], p["size"], p["alpha"], a, p["beta"], r) == 0
            out.append(r)
        return out


def _same(xs, ys):
    return all(np.array_equal(x.view(np.uint8), y.view(np.uint8)) for x, y in zip(xs, ys))


@pytest.fixture(scope="module")
def batch512():
    _say("building the 512-problem batch")
    b = Batch(workloads.batched_problems())
    return b, b.oracle()


def test_batched_512_matches_oracle_and_per_call(batch512):
    import torch
    b, ref = batch512
    b.reset_b()
    h = ttx.ttx_batch_create(b.problems())
    try:
        info = ttx.ttx_batch_get_info(h)
        assert info["count"] == 512 and info["total_tiles"] > 0
        stream = ttx.current_stream()
        ttx.ttx_batch_execute(h, stream)
        got = b.results()
        for i, (g, r, p) in enumerate(zip(got, ref, b.probs)):
            assert_parity(g, r, exact=(p["alpha"] == 1.0 and p["beta"] == 0.0), what="problem %d %s" % (i, p))
        # graph replays, with eager work and synchronisation in between
        for rep in range(3):
            b.reset_b()
            x = torch.ones(1 << 20, device="cuda") * rep
            torch.cuda.synchronize()
            ttx.ttx_batch_execute(h, stream)
            assert _same(b.results(), got), "replay %d differs" % rep
            assert float(x.sum()) == float(rep * (1 << 20))
        # the same persistent kernel without the graph
        b.reset_b()
        ttx.ttx_batch_execute_direct(h, stream)
        assert _same(b.results(), got)
    finally:
        ttx.ttx_batch_destroy(h)
    # the per-call path gives the same bits
    b.reset_b()
    stream = ttx.current_stream()
    for q in b.problems():
        ttx.ttx_transpose(q.dtype, q.n, list(q.perm[:q.n]), list(q.size[:q.n]), None, None, q.alpha,
                          q.A, q.beta, q.B, stream)
    assert _same(b.results(), got)


def test_batched_tuned_is_bitwise_the_same(batch512):
    b, ref = batch512
    sub = Batch(b.probs[:48], seed=100)
    want = ref[:48]
    h = ttx.ttx_batch_create(sub.problems())
    try:
        ttx.ttx_batch_tune(h, 4, 2)
        info = ttx.ttx_batch_get_info(h)
        # problems whose config the tuner replaced (only where a candidate
        # was clearly faster); every problem must compute the same bits
        _say("batch tuning replaced %d of 48 configs" % info["tuned"])
        assert 0 <= info["tuned"] <= 48
        sub.reset_b()
        ttx.ttx_batch_execute(h, ttx.current_stream())
        got = sub.results()
        for g, r, p in zip(got, want, sub.probs):
            assert_parity(g, r, exact=(p["alpha"] == 1.0 and p["beta"] == 0.0))
    finally:
        ttx.ttx_batch_destroy(h)


def test_batch_update_new_pointers():
    import torch
    probs = workloads.batched_problems(count=24, seed=9)
    b1 = Batch(probs, seed=500)
    b2 = Batch(probs, seed=900)
    h = ttx.ttx_batch_create(b1.problems())
    try:
        ttx.ttx_batch_update(h, b2.problems(), ttx.current_stream())
        ttx.ttx_batch_execute(h, ttx.current_stream())
        got = b2.results()
        for g, r, p in zip(got, b2.oracle(), probs):
            assert_parity(g, r, exact=False)
        assert _same(b1.results(), b1.B0)      # the first set was not touched
    finally:
        ttx.ttx_batch_destroy(h)


def test_batch_with_empty_and_degenerate_problems():
    import torch
    probs = [dict(dtype=F32, size=(0, 5), perm=(1, 0), alpha=1.0, beta=0.0),
             dict(dtype=F32, size=(1, 1, 1), perm=(2, 0, 1), alpha=2.0, beta=0.5),
             dict(dtype=np.dtype(np.float64), size=(7, 1, 9), perm=(0, 1, 2), alpha=-1.0, beta=0.25),
             dict(dtype=F32, size=(1000, 3), perm=(1, 0), alpha=1.0, beta=0.0)]
    b = Batch(probs, seed=1)
    h = ttx.ttx_batch_create(b.problems())
    try:
        ttx.ttx_batch_execute(h, ttx.current_stream())
        for g, r in zip(b.results(), b.oracle()):
            assert_parity(g, r, exact=False)
    finally:
        ttx.ttx_batch_destroy(h)
    h = ttx.ttx_batch_create([])
    ttx.ttx_batch_execute(h, ttx.current_stream())
    ttx.ttx_batch_destroy(h)


# -- serving -----------------------------------------------------------------------------
def test_served_results_equal_alone_and_oracle():
    """Requests drawn like the served workload (scaled down), inputs taken from
    a device pool, replayed at 50K requests/s through the server with outputs
    in its arena; sampled results are compared bitwise with the same request
    run alone through ttx_transpose, and with the oracle."""
    import torch
    from gpu_util import dev_copy
    rng = np.random.default_rng(21)
    pool_bytes = 128 << 20
    half = pool_bytes // 2
    host_pool = workloads.uniform(pool_bytes // 4, F32, 22)
    pool = torch.from_numpy(host_pool).cuda()
    raw = host_pool.view(np.uint8)
    times, shapes = workloads.served_trace(rate=50000.0, duration=0.06, seed_arrivals=23, seed_shapes=24,
                                           large_frac=0.02, large_bytes=(4 << 20, 16 << 20))
    n = len(times)
    reqs = ttx._ttx.request_array(n)
    meta = []
    for i, r in enumerate(shapes):
        es = r["dtype"].itemsize
        if workloads.elements(r["size"]) * es > half // 2:     # keep every input inside its half
            r = dict(r, size=(half // 2 // es,), perm=(0,))
        nbytes = workloads.elements(r["size"]) * es
        off_a = int(rng.integers(0, (half - nbytes) // 256 + 1)) * 256
        off_b = half + int(rng.integers(0, (half - nbytes) // 256 + 1)) * 256
        k = len(r["perm"])
        reqs[i]["dtype"] = ttx.F32 if es == 4 else ttx.F64
        reqs[i]["n"] = k
        reqs[i]["perm"][:k] = r["perm"]
        reqs[i]["size"][:k] = r["size"]
        reqs[i]["alpha"] = r["alpha"]
        reqs[i]["beta"] = r["beta"]
        reqs[i]["A"] = pool.data_ptr() + off_a
        reqs[i]["B_in"] = pool.data_ptr() + off_b
        reqs[i]["keep_result"] = 1 if (i % 37 == 0 or r.get("large")) else 0
        meta.append((r, off_a, off_b, nbytes))
    _say("served: %d requests" % n)
    s = ttx.ttx_server_create(slots=4)
    try:
        tickets = ttx.ttx_server_replay(s, reqs, (np.asarray(times) * 1e9).astype(np.int64))
        ttx.ttx_server_drain(s)
        st = ttx.ttx_server_get_stats(s)
        assert st["completed"] == n and st["rejected"] == 0
        assert st["batches"] < n   # requests were batched together
        checked = 0
        stream = ttx.current_stream()
        for i in range(n):
            if not reqs[i]["keep_result"]:
                continue
            r, off_a, off_b, nbytes = meta[i]
            ptr, lat = ttx.ttx_server_result(s, int(tickets[i]))
            assert lat > 0
            ne = workloads.elements(r["size"])
            tdt = _tdt(r["dtype"])
            served = torch.empty(ne, dtype=tdt, device="cuda")
            dev_copy(served.data_ptr(), ptr, nbytes)
            b_in = raw[off_b:off_b + nbytes].view(r["dtype"]).copy()
            alone = torch.from_numpy(b_in).cuda()
            ttx.ttx_transpose(ttx.F32 if r["dtype"].itemsize == 4 else ttx.F64, len(r["perm"]),
                              r["perm"], r["size"], None, None, r["alpha"], pool.data_ptr() + off_a,
                              r["beta"], alone.data_ptr(), stream)
            torch.cuda.synchronize()
            got_alone = alone.cpu().numpy()
            assert np.array_equal(served.cpu().numpy().view(np.uint8), got_alone.view(np.uint8)), i
            a_host = raw[off_a:off_a + nbytes].view(r["dtype"]).copy()
            ref = b_in.copy()
            oracle.transpose(r["perm"], r["size"], r["alpha"], a_host, r["beta"], ref)
            assert_parity(got_alone, ref, exact=False)
            ttx.ttx_server_release(s, int(tickets[i]))
            checked += 1
        assert checked >= 5
        assert ttx.ttx_server_get_stats(s)["in_use_bytes"] == 0
    finally:
        ttx.ttx_server_destroy(s)


def test_served_large_multid_requests_equal_alone_and_oracle():
    """The served workload's large requests at their real size (64..256 MiB,
    N in 3..6, multi-dimensional shapes as drawn) among small ones, replayed
    at 20K requests/s: every large result and every 17th small one is
    compared bitwise with the same request run alone through ttx_transpose,
    and the alone result with the oracle (the first mismatch fails)."""
    import torch
    from gpu_util import dev_copy
    times, shapes = workloads.served_trace(rate=20000.0, duration=0.02, seed_arrivals=31, seed_shapes=32,
                                           large_frac=0.02, large_bytes=(64 << 20, 256 << 20))
    large = [i for i, r in enumerate(shapes) if r["large"]]
    assert len(large) >= 4, "trace holds %d large requests" % len(large)
    large = large[:6]
    small = [i for i, r in enumerate(shapes) if not r["large"]][:120]
    keep = sorted(large + small)
    rng = np.random.default_rng(33)
    pool_bytes = 64 << 20
    host_pool = workloads.uniform(pool_bytes // 4, F32, 34)
    pool = torch.from_numpy(host_pool).cuda()
    raw = host_pool.view(np.uint8)
    half = pool_bytes // 2
    n = len(keep)
    reqs = ttx._ttx.request_array(n)
    meta, owned = [], []
    for slot, i in enumerate(keep):
        r = shapes[i]
        es = r["dtype"].itemsize
        ne = workloads.elements(r["size"])
        nbytes = ne * es
        if r["large"]:   # inputs of their own, kept on the host for the checks
            a_host = workloads.uniform(ne, r["dtype"], 1000 + i)
            b_host = workloads.uniform(ne, r["dtype"], 2000 + i)
            dA = torch.from_numpy(a_host).cuda()
            dB = torch.from_numpy(b_host).cuda()
            owned.append((dA, dB))
            ptr_a, ptr_b = dA.data_ptr(), dB.data_ptr()
        else:
            if nbytes > half // 2:
                r = dict(r, size=(half // 2 // es,), perm=(0,))
                ne = workloads.elements(r["size"])
                nbytes = ne * es
            off_a = int(rng.integers(0, (half - nbytes) // 256 + 1)) * 256
            off_b = half + int(rng.integers(0, (half - nbytes) // 256 + 1)) * 256
            a_host = raw[off_a:off_a + nbytes].view(r["dtype"]).copy()
            b_host = raw[off_b:off_b + nbytes].view(r["dtype"]).copy()
            ptr_a, ptr_b = pool.data_ptr() + off_a, pool.data_ptr() + off_b
        k = len(r["perm"])
        reqs[slot]["dtype"] = ttx.F32 if es == 4 else ttx.F64
        reqs[slot]["n"] = k
        reqs[slot]["perm"][:k] = r["perm"]
        reqs[slot]["size"][:k] = r["size"]
        reqs[slot]["alpha"] = r["alpha"]
        reqs[slot]["beta"] = r["beta"]
        reqs[slot]["A"] = ptr_a
        reqs[slot]["B_in"] = ptr_b
        check = r["large"] or slot % 17 == 0
        reqs[slot]["keep_result"] = 1 if check else 0
        meta.append((r, ptr_a, ptr_b, nbytes, a_host if check else None, b_host if check else None))
    torch.cuda.synchronize()
    _say("served with large requests: %d requests, large %s" %
         (n, [(shapes[i]["size"], shapes[i]["perm"], shapes[i]["dtype"].name) for i in large]))
    offsets = (np.asarray([times[i] for i in keep]) * 1e9).astype(np.int64)
    s = ttx.ttx_server_create(slots=4)
    try:
        tickets = ttx.ttx_server_replay(s, reqs, offsets)
        ttx.ttx_server_drain(s)
        st = ttx.ttx_server_get_stats(s)
        assert st["completed"] == n and st["rejected"] == 0
        stream = ttx.current_stream()
        checked_large = 0
        for slot in range(n):
            if not reqs[slot]["keep_result"]:
                continue
            r, ptr_a, ptr_b, nbytes, a_host, b_host = meta[slot]
            ptr, lat = ttx.ttx_server_result(s, int(tickets[slot]))
            ne = workloads.elements(r["size"])
            served = torch.empty(ne, dtype=_tdt(r["dtype"]), device="cuda")
            dev_copy(served.data_ptr(), ptr, nbytes)
            alone = torch.from_numpy(b_host).cuda()
            ttx.ttx_transpose(ttx.F32 if r["dtype"].itemsize == 4 else ttx.F64, len(r["perm"]), r["perm"],
                              r["size"], None, None, r["alpha"], ptr_a, r["beta"], alone.data_ptr(), stream)
            torch.cuda.synchronize()
            got_alone = alone.cpu().numpy()
            assert np.array_equal(served.cpu().numpy().view(np.uint8), got_alone.view(np.uint8)), \
                ("served differs from alone", slot, r["size"], r["perm"])
            ref = b_host.copy()
            assert oracle.transpose(r["perm"], r["size"], r["alpha"], a_host, r["beta"], ref) == 0
            assert_parity(got_alone, ref, exact=False, what=(slot, r["size"], r["perm"]))
            ttx.ttx_server_release(s, int(tickets[slot]))
            checked_large += int(r["large"])
            del served, alone
        assert checked_large == len(large)
        assert ttx.ttx_server_get_stats(s)["in_use_bytes"] == 0
    finally:
        ttx.ttx_server_destroy(s)


# -- complex and mixed-precision problems in batches and in the server ----------------------
def _typed_problems():
    """(code, A dtype, B dtype, perm, size, alpha, beta) for a mixed list."""
    from gpu_util import C32, C64, F64
    return [
        (ttx.F32, F32, F32, (1, 0), (300, 200), 1.3, 0.7),
        (ttx.C32, C32, C32, (2, 0, 1), (40, 30, 20), 0.5 - 1.25j, 0.25 + 0.5j),
        (ttx.F32_F64, F32, F64, (0, 2, 1), (24, 40, 30), -1.5, 0.0),
        (ttx.C64_C32, C64, C32, (1, 0, 2), (33, 17, 9), 1j, 0j),
        (ttx.F64, F64, F64, (2, 1, 0), (50, 60, 70), 2.0, -1.0),
        (ttx.C64, C64, C64, (0, 1), (1000, 3), 1.0 + 0j, 1.0 + 0j),
        (ttx.F64_F32, F64, F32, (1, 0), (129, 257), 0.75, 0.5),
    ]


class TypedBatch:
    def __init__(self, seed):
        import torch
        from gpu_util import to_device
        self.items = _typed_problems()
        self.A, self.B0, self.dA, self.dB, self.pa, self.pb = [], [], [], [], [], []
        for i, (code, da, db, perm, size, alpha, beta) in enumerate(self.items):
            n = workloads.elements(size)
            a = workloads.uniform(n, da, seed + 2 * i)
            b = workloads.uniform(n, db, seed + 2 * i + 1)
            ta, pa = to_device(a)
            tb, pb = to_device(b)
            self.A.append(a)
            self.B0.append(b)
            self.dA.append(ta)
            self.dB.append(tb)
            self.pa.append(pa)
            self.pb.append(pb)
        torch.cuda.synchronize()

    def problems(self):
        return [ttx.make_problem(code, perm, size, alpha, pa, beta, pb)
                for (code, _, _, perm, size, alpha, beta), pa, pb in zip(self.items, self.pa, self.pb)]

    def reset_b(self):
        import torch
        for d, b in zip(self.dB, self.B0):
            d.copy_(torch.from_numpy(b))
        torch.cuda.synchronize()

    def results(self):
        import torch
        torch.cuda.synchronize()
        return [d.cpu().numpy() for d in self.dB]

    def oracle(self):
        out = []
        for (code, _, _, perm, size, alpha, beta), a, b in zip(self.items, self.A, self.B0):
            r = b.copy()
            assert oracle.transpose(perm, size, alpha, a, beta, r) == 0
            out.append(r)
        return out


def test_batch_with_complex_and_mixed_problems():
    import torch
    tb = TypedBatch(seed=300)
    ref = tb.oracle()
    h = ttx.ttx_batch_create(tb.problems())
    try:
        info = ttx.ttx_batch_get_info(h)
        assert info["count"] == 7 and info["per_call"] == 5   # all but the FP32 and FP64 ones
        stream = ttx.current_stream()
        ttx.ttx_batch_execute(h, stream)
        got = tb.results()
        for g, r, it in zip(got, ref, tb.items):
            assert_parity(g, r, exact=False, what=str(it))
        for rep in range(2):   # graph replays with eager work in between
            tb.reset_b()
            x = torch.ones(1 << 16, device="cuda") * rep
            torch.cuda.synchronize()
            ttx.ttx_batch_execute(h, stream)
            assert _same(tb.results(), got), "replay %d" % rep
            assert float(x.sum()) == float(rep * (1 << 16))
        tb.reset_b()
        ttx.ttx_batch_execute_direct(h, stream)
        assert _same(tb.results(), got)
        # the per-call path gives the same bits
        tb.reset_b()
        for (code, _, _, perm, size, alpha, beta), pa, pb in zip(tb.items, tb.pa, tb.pb):
            ttx.ttx_transpose_c(code, len(perm), perm, size, None, None, alpha, pa, beta, pb, stream)
        assert _same(tb.results(), got)
        # new pointers: the graph is captured again
        tb2 = TypedBatch(seed=700)
        ttx.ttx_batch_update(h, tb2.problems(), stream)
        ttx.ttx_batch_execute(h, stream)
        for g, r in zip(tb2.results(), tb2.oracle()):
            assert_parity(g, r, exact=False)
        ttx.ttx_batch_tune(h, 4, 2)
        tb2.reset_b()
        ttx.ttx_batch_execute(h, stream)
        for g, r in zip(tb2.results(), tb2.oracle()):
            assert_parity(g, r, exact=False)
    finally:
        ttx.ttx_batch_destroy(h)


def test_server_complex_and_mixed_requests_equal_alone():
    tb = TypedBatch(seed=900)
    ref = tb.oracle()
    s = ttx.ttx_server_create(slots=2)
    try:
        tickets = [ttx.ttx_server_submit(s, ttx.make_request(q, 0, False)) for q in tb.problems()]
        ttx.ttx_server_drain(s)
        assert all(ttx.ttx_server_poll(s, t) for t in tickets)
        got = tb.results()
    finally:
        ttx.ttx_server_destroy(s)
    for g, r, it in zip(got, ref, tb.items):
        assert_parity(g, r, exact=False, what=str(it))
    tb.reset_b()
    stream = ttx.current_stream()
    for (code, _, _, perm, size, alpha, beta), pa, pb in zip(tb.items, tb.pa, tb.pb):
        ttx.ttx_transpose_c(code, len(perm), perm, size, None, None, alpha, pa, beta, pb, stream)
    assert _same(tb.results(), got)
