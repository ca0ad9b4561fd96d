"""Host-side logic of batched execution and serving (no GPU): batch planning,
and the server's admission, back-pressure, result holding, draining and
latency accounting, driven by its fake executor (which computes nothing and
touches no memory; requests finish after the time their bytes would take)."""
import time

import numpy as np
import pytest

import paper_1607_01249_amd as ttx
import workloads

FAKE_BASE = 1 << 40


def _fake_problems(probs, gap=256):
    """ttx_problems for workload dicts at made-up, non-overlapping addresses."""
    base = FAKE_BASE
    out = []
    for p in probs:
        nbytes = workloads.elements(p["size"]) * p["dtype"].itemsize
        A = base
        base += nbytes + gap
        B = base
        base += nbytes + gap
        out.append(ttx.make_problem(ttx.F32 if p["dtype"].itemsize == 4 else ttx.F64, p["perm"],
                                    p["size"], p["alpha"], A, p["beta"], B))
    return out


BATCH_SHAPES = {
    (ttx.F32, ttx.FAMILY_MOVED): {(64, 32), (32, 32), (32, 64), (8, 128), (128, 8), (64, 64), (128, 32), (32, 128)},
    (ttx.F64, ttx.FAMILY_MOVED): {(32, 32), (32, 16), (16, 32), (4, 128), (128, 4), (64, 32), (32, 64), (16, 128)},
    # direct preserved tiles, and staged (tile_x, tile_y) for short rows
    (ttx.F32, ttx.FAMILY_PRESERVED): {(64, 16), (16, 64), (8, 8), (4, 4)},
    (ttx.F64, ttx.FAMILY_PRESERVED): {(64, 16), (16, 64), (8, 8), (4, 4)},
    (ttx.F32, ttx.FAMILY_FLAT): {(4096, 1), (1024, 1)},
    (ttx.F64, ttx.FAMILY_FLAT): {(2048, 1), (1024, 1)},
}


def test_batch_plan_uses_the_batched_menu():
    probs = workloads.batched_problems()
    qs = _fake_problems(probs)
    cfgs, tiles = ttx.ttx_batch_plan(qs)
    assert len(cfgs) == 512
    dense = 0
    for q, c, t in zip(qs, cfgs, tiles):
        # the merged row length (kept stride-1 index) of the kept family
        plan = ttx.ttx_plan_create(q.dtype, list(q.perm[:q.n]), list(q.size[:q.n]))
        n0 = ttx.ttx_plan_describe(plan)["size"][0]
        ttx.ttx_plan_destroy(plan)
        if c.flags & ttx.CFG_DENSE:     # dense tiles: run-time extents within the capacity
            dense += 1
            rows = n0 if c.family == ttx.FAMILY_PRESERVED else 1
            assert rows * c.tile_a * c.tile_b * max(1, c.tile_c) <= ttx.DENSE_CAP[q.dtype], c.as_dict()
        else:
            assert (c.tile_a, c.tile_b) in BATCH_SHAPES[(q.dtype, c.family)], c.as_dict()
        assert c.flags & ttx.CFG_XCD_SWIZZLE == 0
        # every element is covered: tiles * tile area >= elements (staged
        # tiles of the kept family also hold whole stride-1 rows)
        n = int(np.prod(list(q.size[:q.n])))
        rows = n0 if (c.family == ttx.FAMILY_PRESERVED and c.group_a > 1) else 1
        assert t >= 1 and t * c.tile_a * max(1, c.tile_b) * max(1, c.tile_c) * rows >= n
    fams = {c.family for c in cfgs}
    assert fams >= {ttx.FAMILY_MOVED, ttx.FAMILY_PRESERVED, ttx.FAMILY_FLAT}
    assert dense > 0


def test_batch_plan_misaligned_pointers_use_scalar_variants():
    q = ttx.make_problem(ttx.F32, (1, 0), (64, 64), 1.0, FAKE_BASE + 4, 0.0, FAKE_BASE + (1 << 20))
    (c,), _ = ttx.ttx_batch_plan([q])
    assert (c.tile_a, c.tile_b) in BATCH_SHAPES[(ttx.F32, ttx.FAMILY_MOVED)]
    q = ttx.make_problem(ttx.F32, (0,), (1001,), 1.0, FAKE_BASE, 0.0, FAKE_BASE + (1 << 20))
    (c,), _ = ttx.ttx_batch_plan([q])
    assert c.family == ttx.FAMILY_FLAT and c.tile_a == 1024    # 1001 % 4 != 0: scalar
    q = ttx.make_problem(ttx.F32, (0,), (1000,), 1.0, FAKE_BASE, 0.0, FAKE_BASE + (1 << 20))
    (c,), _ = ttx.ttx_batch_plan([q])
    assert c.tile_a == 4096


def test_batch_plan_rejects_bad_problems():
    good = ttx.make_problem(ttx.F32, (1, 0), (8, 8), 1.0, FAKE_BASE, 0.0, FAKE_BASE + 4096)
    bad = ttx.make_problem(ttx.F32, (0, 0), (8, 8), 1.0, FAKE_BASE, 0.0, FAKE_BASE + 4096)
    with pytest.raises(ttx.TTXError) as e:
        ttx.ttx_batch_plan([good, bad])
    assert e.value.status == ttx.EPERM
    overlap = ttx.make_problem(ttx.F32, (1, 0), (8, 8), 1.0, FAKE_BASE, 0.0, FAKE_BASE + 16)
    with pytest.raises(ttx.TTXError) as e:
        ttx.ttx_batch_plan([overlap])
    assert e.value.status == ttx.EOVERLAP


def test_static_batch_run_checks_before_any_launch():
    """The allocation-free run refuses too many problems and bad problems
    before it touches a device (so this runs without one)."""
    import re
    hdr = open(__file__.rsplit("/tests/", 1)[0] + "/include/ttx.h").read()
    assert int(re.search(r"#define TTX_STATIC_BATCH_MAX (\d+)", hdr).group(1)) == ttx.STATIC_BATCH_MAX
    good = ttx.make_problem(ttx.F32, (1, 0), (8, 8), 1.0, FAKE_BASE, 0.0, FAKE_BASE + 4096)
    with pytest.raises(ttx.TTXError, match="at most") as e:
        ttx.ttx_batch_run_static([good] * (ttx.STATIC_BATCH_MAX + 1))
    assert e.value.status == ttx.EINVAL
    bad = ttx.make_problem(ttx.F32, (0, 0), (8, 8), 1.0, FAKE_BASE, 0.0, FAKE_BASE + 4096)
    with pytest.raises(ttx.TTXError) as e:
        ttx.ttx_batch_run_static([good, bad])
    assert e.value.status == ttx.EPERM


# -- server with the fake executor -------------------------------------------------------
def _req(size=(64, 64), perm=(1, 0), dtype=ttx.F32, beta=0.0, A=FAKE_BASE, B=None, B_in=None,
         keep=False):
    q = ttx.make_problem(dtype, perm, size, 1.5, A, beta, B, B_in=B_in)
    return ttx.make_request(q, 0, keep)


def test_server_budget_rejects_oversized_request():
    s = ttx.ttx_server_create(fake_device=True, fake_free_bytes=1 << 20)   # budget 0.8 MiB
    try:
        with pytest.raises(ttx.TTXError) as e:
            ttx.ttx_server_submit(s, _req(size=(512, 512)))   # 1 MiB in + 1 MiB out
        assert e.value.status == ttx.EBUSY
        t = ttx.ttx_server_submit(s, _req(size=(64, 64)))
        ttx.ttx_server_wait(s, t)
        st = ttx.ttx_server_get_stats(s)
        assert st["rejected"] == 1 and st["completed"] == 1 and st["in_use_bytes"] == 0
    finally:
        ttx.ttx_server_destroy(s)


def test_server_holds_results_until_release_and_blocks_admission():
    # each request: 64 KiB in + 64 KiB out; budget 0.8 * 512 KiB -> 3 fit
    s = ttx.ttx_server_create(fake_device=True, fake_free_bytes=512 << 10, max_queue=4)
    try:
        held = [ttx.ttx_server_submit(s, _req(size=(128, 128), keep=True)) for _ in range(3)]
        for t in held:
            ttx.ttx_server_wait(s, t)
        st = ttx.ttx_server_get_stats(s)
        assert st["in_use_bytes"] == 3 * 2 * 65536
        blocked = [ttx.ttx_server_submit(s, _req(size=(128, 128))) for _ in range(4)]
        time.sleep(0.05)
        assert not any(ttx.ttx_server_poll(s, t) for t in blocked)
        with pytest.raises(ttx.TTXError) as e:      # queue of 4 is full
            ttx.ttx_server_submit(s, _req(size=(128, 128)))
        assert e.value.status == ttx.EBUSY
        with pytest.raises(ttx.TTXError) as e:      # nothing running, head cannot be admitted
            ttx.ttx_server_drain(s)
        assert e.value.status == ttx.EBUSY
        ptr, lat = ttx.ttx_server_result(s, held[0])
        assert ptr >= 1 << 44 and lat >= 0
        for t in held:
            ttx.ttx_server_release(s, t)
        ttx.ttx_server_drain(s)
        assert all(ttx.ttx_server_poll(s, t) for t in blocked)
        with pytest.raises(ttx.TTXError) as e:
            ttx.ttx_server_release(s, held[0])
        assert e.value.status == ttx.ENOTFOUND
        st = ttx.ttx_server_get_stats(s)
        assert st["completed"] == 7 and st["in_use_bytes"] == 0
        assert st["peak_in_use_bytes"] <= st["budget_bytes"]
    finally:
        ttx.ttx_server_destroy(s)


def test_server_validation():
    s = ttx.ttx_server_create(fake_device=True)
    try:
        with pytest.raises(ttx.TTXError) as e:     # beta != 0 with an arena output needs B_in
            ttx.ttx_server_submit(s, _req(beta=0.5))
        assert e.value.status == ttx.EINVAL
        with pytest.raises(ttx.TTXError) as e:
            ttx.ttx_server_submit(s, _req(perm=(0, 0)))
        assert e.value.status == ttx.EPERM
        t = ttx.ttx_server_submit(s, _req(beta=0.5, B_in=FAKE_BASE + (1 << 20)))
        ttx.ttx_server_wait(s, t)
        with pytest.raises(ttx.TTXError):
            ttx.ttx_server_poll(s, 12345)
    finally:
        ttx.ttx_server_destroy(s)


def test_server_replay_batches_and_accounts_latency():
    n = 3000
    reqs = ttx._ttx.request_array(n)
    rng = np.random.default_rng(3)
    for i in range(n):
        k = int(rng.integers(2, 5))
        reqs[i]["dtype"] = ttx.F32 if rng.random() < 0.7 else ttx.F64
        reqs[i]["n"] = k
        reqs[i]["perm"][:k] = rng.permutation(k)
        reqs[i]["size"][:k] = rng.integers(2, 40, size=k)
        reqs[i]["alpha"] = 1.0
        reqs[i]["beta"] = 0.0
        reqs[i]["A"] = FAKE_BASE
    offsets = np.cumsum(np.random.default_rng(4).exponential(1e9 / 100000.0, size=n)).astype(np.int64)
    s = ttx.ttx_server_create(fake_device=True, slots=2, max_batch=64)
    try:
        tickets = ttx.ttx_server_replay(s, reqs, offsets)
        assert (tickets > 0).all() and len(set(tickets.tolist())) == n
        ttx.ttx_server_drain(s)
        st = ttx.ttx_server_get_stats(s)
        assert st["submitted"] == n and st["completed"] == n and st["rejected"] == 0
        assert 0 <= st["p50_us"] <= st["p99_us"] <= st["max_us"]
        assert st["batches"] <= n and st["mean_batch"] >= 1.0
        assert st["span_s"] >= offsets[-1] * 1e-9 * 0.99
        assert st["in_use_bytes"] == 0
    finally:
        ttx.ttx_server_destroy(s)


def test_server_destroy_with_queued_work():
    s = ttx.ttx_server_create(fake_device=True, fake_free_bytes=256 << 10)
    t = ttx.ttx_server_submit(s, _req(size=(128, 128), keep=True))
    ttx.ttx_server_wait(s, t)
    for _ in range(5):
        ttx.ttx_server_submit(s, _req(size=(128, 128)))
    ttx.ttx_server_destroy(s)   # must return although the queue is blocked


def test_server_runs_large_requests_alone():
    # 64 MiB in + 64 MiB out: at least 32 MiB of traffic, so it takes a slot by itself
    s = ttx.ttx_server_create(fake_device=True, fake_free_bytes=1 << 34, slots=2)
    try:
        small = [ttx.ttx_server_submit(s, _req(size=(64, 64))) for _ in range(3)]
        big = ttx.ttx_server_submit(s, _req(size=(4096, 4096)))
        more = [ttx.ttx_server_submit(s, _req(size=(64, 64))) for _ in range(3)]
        ttx.ttx_server_drain(s)
        st = ttx.ttx_server_get_stats(s)
        assert st["completed"] == 7 and st["in_use_bytes"] == 0
        assert st["batches"] >= 2     # the large request never shares a micro-batch
        assert all(ttx.ttx_server_poll(s, t) for t in small + [big] + more)
    finally:
        ttx.ttx_server_destroy(s)


def test_server_replay_from_several_clients():
    n = 2000
    reqs = ttx._ttx.request_array(n)
    rng = np.random.default_rng(5)
    for i in range(n):
        k = int(rng.integers(2, 5))
        reqs[i]["dtype"] = ttx.F32
        reqs[i]["n"] = k
        reqs[i]["perm"][:k] = rng.permutation(k)
        reqs[i]["size"][:k] = rng.integers(2, 30, size=k)
        reqs[i]["alpha"] = 1.0
        reqs[i]["A"] = FAKE_BASE
    s = ttx.ttx_server_create(fake_device=True, slots=4)
    try:
        tickets = ttx.ttx_server_replay_clients(s, reqs, np.zeros(n, dtype=np.int64), 4)
        assert (tickets > 0).all() and len(set(tickets.tolist())) == n
        ttx.ttx_server_drain(s)
        st = ttx.ttx_server_get_stats(s)
        assert st["submitted"] == n and st["completed"] == n and st["in_use_bytes"] == 0
    finally:
        ttx.ttx_server_destroy(s)
    with pytest.raises(ttx.TTXError):
        s = ttx.ttx_server_create(fake_device=True)
        try:
            ttx.ttx_server_replay_clients(s, reqs[:4], np.zeros(4, dtype=np.int64), 0)
        finally:
            ttx.ttx_server_destroy(s)


def test_server_runs_complex_and_mixed_requests_alone():
    """Complex and mixed-precision requests take the per-call path (a slot of
    their own), whatever their size; real scalars only for real types."""
    s = ttx.ttx_server_create(fake_device=True, fake_free_bytes=1 << 34, slots=2)
    try:
        tickets = []
        for code, alpha in ((ttx.C64, 0.5 - 2j), (ttx.F32_F64, 1.5), (ttx.C32_C64, 1j)):
            q = ttx.make_problem(code, (1, 0), (64, 64), alpha, FAKE_BASE, 0.0, FAKE_BASE + (1 << 20))
            tickets.append(ttx.ttx_server_submit(s, ttx.make_request(q, 0, False)))
            tickets.append(ttx.ttx_server_submit(s, _req(size=(64, 64))))
        ttx.ttx_server_drain(s)
        st = ttx.ttx_server_get_stats(s)
        assert st["completed"] == 6 and st["batches"] >= 4
        assert all(ttx.ttx_server_poll(s, t) for t in tickets)
        bad = ttx.make_problem(ttx.F64, (1, 0), (64, 64), 1j, FAKE_BASE, 0.0, FAKE_BASE + (1 << 20))
        with pytest.raises(ttx.TTXError) as e:
            ttx.ttx_server_submit(s, ttx.make_request(bad, 0, False))
        assert e.value.status == ttx.EINVAL
    finally:
        ttx.ttx_server_destroy(s)


def test_server_cancel_withdraws_queued_requests_only():
    """A request held back by admission is withdrawn and never runs; a
    running or finished request cannot be cancelled; a cancelled ticket is
    unknown afterwards; the budget and the rest of the queue are unaffected."""
    # each request: 64 KiB in + 64 KiB out; budget 0.8 * 512 KiB -> 3 fit
    s = ttx.ttx_server_create(fake_device=True, fake_free_bytes=512 << 10, max_queue=8)
    try:
        held = [ttx.ttx_server_submit(s, _req(size=(128, 128), keep=True)) for _ in range(3)]
        for t in held:
            ttx.ttx_server_wait(s, t)
        queued = [ttx.ttx_server_submit(s, _req(size=(128, 128))) for _ in range(3)]
        time.sleep(0.02)
        ttx.ttx_server_cancel(s, queued[1])
        for call in (lambda: ttx.ttx_server_poll(s, queued[1]), lambda: ttx.ttx_server_wait(s, queued[1]),
                     lambda: ttx.ttx_server_result(s, queued[1]), lambda: ttx.ttx_server_release(s, queued[1]),
                     lambda: ttx.ttx_server_cancel(s, queued[1]), lambda: ttx.ttx_server_cancel(s, 10 ** 6)):
            with pytest.raises(ttx.TTXError) as e:
                call()
            assert e.value.status == ttx.ENOTFOUND
        with pytest.raises(ttx.TTXError) as e:      # finished: released, not cancelled
            ttx.ttx_server_cancel(s, held[0])
        assert e.value.status == ttx.EBUSY
        for t in held:
            ttx.ttx_server_release(s, t)
        ttx.ttx_server_drain(s)
        assert ttx.ttx_server_poll(s, queued[0]) and ttx.ttx_server_poll(s, queued[2])
        st = ttx.ttx_server_get_stats(s)
        assert st["completed"] == 5 and st["queued"] == 0 and st["in_use_bytes"] == 0
        ttx.ttx_server_drain(s)
    finally:
        ttx.ttx_server_destroy(s)


def test_server_cancel_refuses_a_launched_request():
    """The fake executor holds a request for bytes / 4 TB/s: an FP64
    65536 x 65536 transposition (68.7 GB of traffic) runs for about 17 ms.
    Once the server counts it as running (or finished), cancelling it is
    refused."""
    s = ttx.ttx_server_create(fake_device=True, fake_free_bytes=1 << 40)
    try:
        big = ttx.ttx_server_submit(s, _req(size=(65536, 65536), dtype=ttx.F64))
        t0 = time.time()
        while True:
            st = ttx.ttx_server_get_stats(s)
            if st["running"] or st["completed"]:
                break
            assert time.time() - t0 < 10, "the dispatcher never launched the request"
            time.sleep(0.0002)
        with pytest.raises(ttx.TTXError) as e:
            ttx.ttx_server_cancel(s, big)
        assert e.value.status == ttx.EBUSY
        ttx.ttx_server_wait(s, big)
        assert ttx.ttx_server_get_stats(s)["completed"] == 1
    finally:
        ttx.ttx_server_destroy(s)
