"""GPU parity for size-specialised kernels (compiled at run time with hipRTC,
the problem's sizes and strides as constants; Sec. 2.1), through the C ABI:
bit-identical with the generic kernels and with the CPU oracle to the same
bar (bit-exact for alpha = 1, beta = 0; at most 1 ulp otherwise)."""
import os
import sys

import numpy as np
import pytest

import oracle
import paper_1607_01249_amd as ttx
import workloads
from gpu_util import C32, C64, F32, F64, assert_parity, dtype_code, gpu_transpose

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _scalars(db, beta_zero):
    if db in (C32, C64):
        return complex(0.75, -1.25), (0j if beta_zero else complex(-0.5, 0.375))
    return 1.3, (0.0 if beta_zero else 0.7)


def _inputs(perm, size, da, db, seed, outer_a=None, outer_b=None):
    size_b = [size[p] for p in perm]
    A = workloads.uniform(workloads.elements(outer_a or size), da, seed=9000 + seed) * 3
    B = workloads.uniform(workloads.elements(outer_b or size_b), db, seed=9500 + seed)
    return A, B


def _check(perm, size, da, db, beta_zero, seed=0, outer_a=None, outer_b=None, plan_config=None, pad_a=0,
           pad_b=0):
    alpha, beta = _scalars(db, beta_zero)
    A, B = _inputs(perm, size, da, db, seed, outer_a, outer_b)
    ref = B.copy()
    assert oracle.transpose(perm, size, alpha, A, beta, ref, outer_a, outer_b) == 0
    got = gpu_transpose(perm, size, alpha, A, beta, B, outer_a, outer_b, pad_a, pad_b, plan_config,
                        specialise=True)
    generic = gpu_transpose(perm, size, alpha, A, beta, B, outer_a, outer_b, pad_a, pad_b, plan_config)
    assert np.array_equal(got.view(np.uint8), generic.view(np.uint8)), (perm, size, "differs from generic")
    assert_parity(got, ref, alpha == 1 and beta == 0, (perm, size))


TYPES = [(F32, F32), (F64, F64), (C32, C32), (C64, C64), (F32, F64), (F64, F32), (C32, C64), (C64, C32)]
TYPE_IDS = ["s", "d", "c", "z", "sd", "ds", "cz", "zc"]
SHAPES = [((2, 0, 3, 1), (37, 70, 19, 23)), ((2, 1, 0), (33, 40, 27)), ((0, 2, 1), (64, 9, 48)),
          ((0, 5, 1, 4, 2, 3), (5, 7, 6, 4, 3, 5)), ((0, 2, 1, 3), (40, 9, 11, 13)), ((1, 0, 2), (3, 4, 700)),
          ((4, 3, 2, 1, 0), (13, 17, 11, 9, 7))]


@pytest.mark.parametrize("beta_zero", [False, True], ids=["beta", "beta0"])
@pytest.mark.parametrize("types", TYPES, ids=TYPE_IDS)
def test_specialised_matches_generic_and_oracle(types, beta_zero):
    da, db = types
    for i, (perm, size) in enumerate(SHAPES):
        _check(perm, size, da, db, beta_zero, seed=i)


PER_KIND = 5


@pytest.mark.parametrize("dtype", [F32, F64, C64])
@pytest.mark.parametrize("perm,size", [((2, 0, 3, 1), (37, 70, 19, 23)), ((0, 2, 1, 3), (40, 9, 11, 13)),
                                       ((0, 2, 1), (5, 40, 33)), ((1, 0, 2), (3, 4, 700)),
                                       ((0, 5, 1, 4, 2, 3), (24, 7, 4, 3, 5, 6))])
def test_every_tile_kind_specialised(perm, size, dtype):
    """Distinct tiles of every tile kind (menu, staged, dense, whole-unit
    dense), the best-ranked PER_KIND of each, each specialised: the same
    bits as its generic kernel.  (Every kernel is compiled at run time; the
    bound keeps the test to a few dozen compilations.)"""
    cands, _ = ttx.ttx_tune_candidates(dtype_code(dtype), perm, size, max_candidates=-1, cap=200000)
    seen, pick, per_kind = set(), [], {}
    for c in cands:
        key = (c.tile_a, c.tile_b, c.group_a, c.group_b, c.tile_c, c.flags & (ttx.CFG_DENSE | ttx.CFG_WIDE))
        kind = (c.family, c.flags & (ttx.CFG_DENSE | ttx.CFG_WIDE), c.group_a > 1 or c.group_b > 1)
        if key not in seen and per_kind.get(kind, 0) < PER_KIND:
            seen.add(key)
            per_kind[kind] = per_kind.get(kind, 0) + 1
            pick.append(c)
    _say("specialised candidates %s %s %s: %d configs" % (perm, size, np.dtype(dtype).name, len(pick)))
    for bz in (False, True):
        for c in pick:
            _check(perm, size, dtype, dtype, bz, seed=3, plan_config=c)


EDGE = [((1, 0), (1, 1), None, None), ((3, 2, 1, 0), (5, 3, 7, 9), (6, 3, 8, 9), (10, 7, 3, 5)),
        ((0, 2, 1), (6, 50, 40), (8, 52, 41), (7, 41, 51)), ((1, 0, 2), (3, 4, 700), (4, 5, 700), (5, 3, 701)),
        ((5, 4, 3, 2, 1, 0), (7, 5, 3, 6, 5, 3), None, None), ((2, 0, 1), (3, 1, 200), None, None)]


@pytest.mark.parametrize("perm,size,oa,ob", EDGE)
@pytest.mark.parametrize("dtype", [F32, F64])
def test_edge_and_leading_dimension_shapes(perm, size, oa, ob, dtype):
    for bz in (False, True):
        _check(perm, size, dtype, dtype, bz, seed=5, outer_a=oa, outer_b=ob)


@pytest.mark.parametrize("pad_a,pad_b", [(1, 0), (0, 1), (1, 3)])
def test_misaligned_pointers_fall_back(pad_a, pad_b):
    """Pointers outside the vector alignment the kernel was compiled for run
    the generic kernel (whole-unit dense tiles need unit-aligned rows)."""
    for perm, size in [((0, 5, 1, 4, 2, 3), (24, 7, 4, 3, 5, 6)), ((2, 1, 0), (64, 9, 48)),
                       ((0, 2, 1), (64, 9, 48))]:
        _check(perm, size, F32, F32, False, seed=8, pad_a=pad_a, pad_b=pad_b)


def test_flat_and_empty_attach_nothing():
    for perm, size in [((0, 1), (64, 9)), ((0,), (1000,)), ((1, 0), (1, 0))]:
        plan = ttx.ttx_plan_create(ttx.F32, perm, size)
        try:
            ttx.ttx_plan_specialise(plan, True)
            assert ttx.ttx_plan_describe(plan)["specialised"] == [0, 0]
        finally:
            ttx.ttx_plan_destroy(plan)


def test_set_config_drops_the_specialised_kernel():
    perm, size = (2, 0, 1), (40, 30, 20)
    plan = ttx.ttx_plan_create(ttx.F64, perm, size)
    try:
        ttx.ttx_plan_specialise(plan, False)
        ttx.ttx_plan_specialise(plan, True)
        assert ttx.ttx_plan_describe(plan)["specialised"] == [1, 1]
        cfg = ttx.ttx_plan_describe(plan)["config_raw"][0]
        ttx.ttx_plan_set_config(plan, False, cfg)
        assert ttx.ttx_plan_describe(plan)["specialised"] == [0, 1]
    finally:
        ttx.ttx_plan_destroy(plan)


def test_timed_specialisation_keeps_the_faster_kernel():
    """reps > 0 times both kernels and attaches the specialised one only when
    it wins; either way the plan computes the same bits."""
    for perm, size, bz in [((0, 5, 1, 4, 2, 3), (20, 16, 16, 20, 16, 16), False),
                           ((2, 0, 3, 1), (160, 160, 32, 32), True), ((0, 2, 1), (64, 90, 48), False)]:
        plan = ttx.ttx_plan_create(ttx.F64, perm, size)
        try:
            kept = ttx.ttx_plan_specialise(plan, bz, reps=3)
            assert ttx.ttx_plan_describe(plan)["specialised"][int(bz)] == int(kept)
            _say("timed specialisation %s %s beta0=%s: kept=%s" % (perm, size, bz, kept))
        finally:
            ttx.ttx_plan_destroy(plan)
        _check(perm, size, F64, F64, bz, seed=12)


def test_kernel_name_names_the_specialised_kernel():
    import torch
    plan = ttx.ttx_plan_create(ttx.F32, (2, 0, 3, 1), (37, 70, 19, 23))
    try:
        generic = ttx.ttx_plan_kernel_name(plan, 0.7, 1 << 20, 3 << 20)
        assert generic.startswith("k_moved<float, false")
        ttx.ttx_plan_specialise(plan, False)
        name = ttx.ttx_plan_kernel_name(plan, 0.7, 1 << 20, 3 << 20)
        assert name.startswith("ttx_jit_moved_float_b_"), name
        assert ttx.ttx_plan_kernel_name(plan, 0.0, 1 << 20, 3 << 20).startswith("k_moved<float, true")
    finally:
        ttx.ttx_plan_destroy(plan)


@pytest.mark.parametrize("dtype,perm,size,bz", [(F64, (2, 0, 1), (40, 30, 20), False),
                                              (F32, (0, 5, 1, 4, 2, 3), (24, 7, 4, 3, 5, 6), True),
                                              (F32, (0, 1), (64, 9), False)])
def test_tune_specialised_stores_a_config(dtype, perm, size, bz):
    """Candidates compiled and timed as specialised kernels: the winner lands
    in the tune table, and the plan that takes it computes the oracle's bits."""
    code = dtype_code(dtype)
    best, timed = ttx.ttx_tune_specialised(code, perm, size, beta_is_zero=bz, max_candidates=6, reps=2)
    assert timed >= 1
    plan = ttx.ttx_plan_create(code, perm, size)
    try:
        info = ttx.ttx_plan_describe(plan)
        if info["family"] in ("moved", "preserved"):
            ttx.ttx_plan_specialise(plan, bz)   # takes the entry for specialised execution
            info = ttx.ttx_plan_describe(plan)
            assert info["config_from_table"][int(bz)] == 1 and info["specialised"][int(bz)] == 1
        else:   # single-index problems take the generic search and entry
            assert info["config_from_table"][int(bz)] == 1
        assert info["config"][int(bz)] == best.as_dict()
    finally:
        ttx.ttx_plan_destroy(plan)
    _check(perm, size, dtype, dtype, bz, seed=13)


def test_auto_specialise_hot_shapes():
    """With automatic specialisation at the 3rd call, a shape called through
    ttx_transpose gets its specialised kernel then, and every call computes
    the oracle's bits."""
    perm, size = (3, 1, 0, 2), (23, 29, 6, 7)   # a shape no other test calls
    A, B = _inputs(perm, size, F32, F32, 21)
    ref = B.copy()
    oracle.transpose(perm, size, 1.3, A, 0.7, ref)
    ttx.ttx_set_auto_specialise(3)
    try:
        before = ttx.ttx_transpose_cache_info()[1]
        for k in range(4):
            got = gpu_transpose(perm, size, 1.3, A, 0.7, B)
            assert_parity(got, ref, False, k)
            assert ttx.ttx_transpose_cache_info()[1] == before + (1 if k >= 2 else 0), k
    finally:
        ttx.ttx_set_auto_specialise(0)


def test_disk_cache_written_and_reused(tmp_path):
    """With TTX_JIT_CACHE set, the code object lands in the directory; a
    second process finds it there and leaves it untouched."""
    import subprocess
    d = tmp_path / "jit"
    perm, size = (2, 0, 3, 1), (29, 31, 7, 5)   # not compiled elsewhere in this process
    os.environ["TTX_JIT_CACHE"] = str(d)
    try:
        _check(perm, size, F32, F32, False, seed=11)
    finally:
        del os.environ["TTX_JIT_CACHE"]
    files = sorted(os.listdir(d))
    assert len(files) == 1 and files[0].endswith(".co"), files
    mtime = os.stat(d / files[0]).st_mtime_ns
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = ("import sys; sys.path.insert(0, %r); import paper_1607_01249_amd as ttx\n"
            "p = ttx.ttx_plan_create(ttx.F32, %r, %r); ttx.ttx_plan_specialise(p, False)\n"
            "assert ttx.ttx_plan_describe(p)['specialised'][0] == 1; print('reused')" % (root, perm, size))
    env = dict(os.environ, TTX_JIT_CACHE=str(d))
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    assert sorted(os.listdir(d)) == files and os.stat(d / files[0]).st_mtime_ns == mtime
    # a damaged file (not an ELF image: the host loader rejects it) is compiled again and replaced
    (d / files[0]).write_bytes(b"damaged code object")
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    assert sorted(os.listdir(d)) == files and (d / files[0]).read_bytes()[:4] == b"\x7fELF"


# -- full sizes (about 200 MiB per tensor): the cases the throughput figures time ------------
@pytest.mark.parametrize("dtype,perm,beta_zero", [(F64, (2, 0, 3, 1), False), (F32, (3, 2, 1, 0), True),
                                                   (F32, (0, 5, 1, 4, 2, 3), True),
                                                   (F64, (0, 5, 1, 4, 2, 3), False),
                                                   (F64, (1, 3, 0, 4, 2), True)])
def test_full_size_specialised(dtype, perm, beta_zero):
    rank = "%dd" % len(perm)
    size = workloads.LARGE_SHAPES[(rank, dtype)]
    _say("full-size specialised %s %s %s beta0=%s" % (np.dtype(dtype).name, perm, size, beta_zero))
    _check(perm, size, dtype, dtype, beta_zero, seed=30)


@pytest.mark.parametrize("code,perm,size", [
    (ttx.F32, (3, 2, 1, 0), (150, 7, 13, 140)), (ttx.F64, (2, 1, 0), (200, 9, 131)),
    (ttx.C64, (1, 0, 2), (70, 66, 3)), (ttx.F32_F64, (4, 3, 2, 1, 0), (33, 5, 6, 7, 90))])
def test_large_run_time_tiles_match_the_oracle(code, perm, size):
    """Every run-time-only large moved tile (each compiled at run time), at
    256 and 512 threads with line-aligned A runs on and off, ragged at both
    tile edges: the oracle's bits at both beta classes."""
    from gpu_util import TYPES_OF_CODE
    da, db = TYPES_OF_CODE[code]
    n = workloads.elements(size)
    A = workloads.uniform(n, da, 40)
    B = workloads.uniform(n, db, 41)
    plan = ttx.ttx_plan_create(code, perm, size)
    try:
        base = ttx.Config.from_buffer_copy(ttx.ttx_plan_describe(plan)["config_raw"][0])
    finally:
        ttx.ttx_plan_destroy(plan)
    assert base.family == ttx.FAMILY_MOVED
    cx = db in (C32, C64)
    for k, shape in enumerate(ttx.ttx_tile_shapes(code, ttx.FAMILY_MOVED, run_time_only=True)):
        c = ttx.Config.from_buffer_copy(base)
        c.tile_a, c.tile_b, c.threads, c.lds_pad = shape[0], shape[1], (256, 512)[k % 2], 1
        c.flags &= ~(ttx.CFG_DENSE | ttx.CFG_WIDE | ttx.CFG_ALIGN_A)
        for beta in ((0.5 - 0.25j, 0j) if cx else (0.7, 0.0)):
            alpha = (1.25 + 0.5j) if cx else 1.3
            ref = B.copy()
            assert oracle.transpose(perm, size, alpha, A, beta, ref) == 0
            for align in (0, ttx.CFG_ALIGN_A):
                c.flags = (c.flags & ~ttx.CFG_ALIGN_A) | align
                _say("large %s align=%d beta=%s" % (shape, align, beta))
                try:
                    got = gpu_transpose(perm, size, alpha, A, beta, B, plan_config=c)
                except ttx.TTXError:
                    assert align, "the large tile itself must be valid"
                    continue   # line-aligned runs need a contiguous A run along the tile
                assert_parity(got, ref, exact=True, what="%s %s" % (shape, c.as_dict()))


@pytest.mark.parametrize("code,perm,size", [
    (ttx.F32, (1, 0, 2), (3000, 3001, 3)), (ttx.F64, (2, 1, 0), (301, 40, 2500)),
    (ttx.F32, (0, 2, 1, 3), (40, 90, 70, 13)), (ttx.F64, (0, 5, 1, 4, 2, 3), (20, 7, 4, 3, 5, 6)),
    (ttx.C64, (2, 1, 0), (33, 40, 27)), (ttx.F32_F64, (3, 2, 1, 0), (5, 3, 70, 9))])
def test_pipelined_grids_match_the_oracle(code, perm, size):
    """TTX_CFG_PIPELINED (a resident grid whose workgroups loop over tiles,
    loading the next tile before storing the current one) on the two
    best-ranked candidates of each tile kind but dense, at 256 and 512
    threads (moved tiles also with line-aligned A runs): the oracle's bits
    at both beta classes.  The first two problems have several tiles per
    resident workgroup."""
    from gpu_util import TYPES_OF_CODE
    da, db = TYPES_OF_CODE[code]
    cands, _ = ttx.ttx_tune_candidates(code, perm, size, max_candidates=-1, cap=200000)
    per_kind, picks = {}, []
    for c in cands:
        if c.flags & ttx.CFG_DENSE:
            continue
        kind = (c.family, c.group_a > 1 or c.group_b > 1)
        if per_kind.get(kind, 0) < 2:
            per_kind[kind] = per_kind.get(kind, 0) + 1
            picks.append(c)
    n = workloads.elements(size)
    A = workloads.uniform(n, da, 50)
    B = workloads.uniform(n, db, 51)
    cx = db in (C32, C64)
    for beta in ((0.5 - 0.25j, 0j) if cx else (0.7, 0.0)):
        alpha = (1.25 + 0.5j) if cx else 1.3
        ref = B.copy()
        assert oracle.transpose(perm, size, alpha, A, beta, ref) == 0
        for k, base in enumerate(picks):
            c = ttx.Config.from_buffer_copy(base)
            c.flags |= ttx.CFG_PIPELINED
            c.threads = (256, 512)[k % 2]
            if c.family == ttx.FAMILY_MOVED and k % 2:
                c.flags |= ttx.CFG_ALIGN_A
            _say("pipelined %s beta=%s" % (c.as_dict(), beta))
            try:
                got = gpu_transpose(perm, size, alpha, A, beta, B, plan_config=c)
            except ttx.TTXError:
                assert c.threads != 256 or c.flags & ttx.CFG_ALIGN_A, "the base config must stay valid"
                continue   # the tile does not fit 512 threads, or no contiguous A run to align
            assert_parity(got, ref, exact=True, what=str(c.as_dict()))
