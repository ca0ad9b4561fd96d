"""GPU parity: the HIP library (through its C ABI) against the CPU oracle.

Bit-exact for alpha = 1, beta = 0; at most 1 ulp otherwise (both sides
evaluate fl(fl(alpha*a) + fl(beta*b)) with no fused multiply-add, so
bit-identity is the expectation there too and the number of differing
elements is reported).
"""
import itertools
import os
import sys

import numpy as np
import pytest

import oracle
import paper_1607_01249_amd as ttx
import workloads
from gpu_util import F32, F64, assert_parity, from_device, gpu_transpose, to_device

pytestmark = pytest.mark.gpu


def _elems(d):
    return workloads.elements(d)


def _case(perm, size, dtype, alpha, beta, outer_a=None, outer_b=None, seed=0, pad_a=0, pad_b=0,
          plan_config=None, B_fill=None):
    size_b = [size[p] for p in perm]
    A = workloads.uniform(_elems(outer_a or size), dtype, seed=1000 + seed)
    if B_fill is None:
        B = workloads.uniform(_elems(outer_b or size_b), dtype, seed=2000 + seed)
    else:
        B = np.full(_elems(outer_b or size_b), B_fill, dtype=dtype)
    ref = B.copy()
    assert oracle.transpose(perm, size, alpha, A, beta, ref, outer_a, outer_b) == 0
    got = gpu_transpose(perm, size, alpha, A, beta, B, outer_a, outer_b, pad_a, pad_b, plan_config)
    exact = alpha == 1.0 and beta == 0.0
    return got, ref, exact


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


# -- configuration 1: the plain correctness case ----------------------------------------
def test_plain_3d_f32_bit_exact():
    c = workloads.PLAIN
    n = _elems(c["size"])
    A = workloads.uniform(n, c["dtype"], c["seed_a"])
    B = np.zeros(n, dtype=c["dtype"])
    ref = B.copy()
    assert oracle.transpose(c["perm"], c["size"], 1.0, A, 0.0, ref) == 0
    got = gpu_transpose(c["perm"], c["size"], 1.0, A, 0.0, B)
    assert_parity(got, ref, exact=True)


# -- paper-shaped permutations at reduced sizes (several tiles, ragged edges) -----------
REDUCED = {"4d": (37, 70, 19, 23), "5d": (13, 17, 11, 9, 7), "6d": (5, 7, 6, 4, 3, 5)}
REDUCED_CASES = [(rank, perm, dt, beta) for rank in ("4d", "5d", "6d")
                 for perm in workloads.LARGE_PERMS[rank] for dt in (F32, F64) for beta in (0.7, 0.0)]


@pytest.mark.parametrize("rank,perm,dtype,beta", REDUCED_CASES)
def test_reduced_large_perms(rank, perm, dtype, beta):
    got, ref, exact = _case(perm, REDUCED[rank], dtype, 1.3, beta, seed=3)
    assert_parity(got, ref, exact, (rank, perm, dtype, beta))


@pytest.mark.parametrize("rank,perm,dtype", [(r, p, d) for r in ("4d", "5d", "6d")
                                             for p in workloads.LARGE_PERMS[r] for d in (F32, F64)])
def test_reduced_large_perms_plain_copy_exact(rank, perm, dtype):
    got, ref, exact = _case(perm, REDUCED[rank], dtype, 1.0, 0.0, seed=4)
    assert exact
    assert_parity(got, ref, True)


# -- paper-shaped permutations at full size (about 200 MiB per tensor) -------------------
# These run the kernels the throughput step times: the shipped tune table is
# loaded, and each case runs (a) through ttx_transpose (the generic kernel
# with the table's configuration) and (b) through a plan with its
# size-specialised kernel (the table's configuration for specialised
# execution where it has one), both against the oracle on every element.
TABLE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                     "paper_1607_01249_amd", "tune", "gfx950.txt")


@pytest.fixture(scope="module")
def shipped_table():
    ttx.ttx_tune_table_clear()
    ttx.ttx_tune_table_load(TABLE)
    yield
    ttx.ttx_tune_table_clear()


@pytest.mark.parametrize("case", workloads.large_cases(), ids=lambda c: c["name"])
def test_full_size_large_perms(case, shipped_table):
    import torch
    _say("full-size case %s" % case["name"])
    perm, size, dtype = case["perm"], case["size"], case["dtype"]
    code = ttx.F32 if dtype == F32 else ttx.F64
    n = _elems(size)
    A = workloads.uniform(n, dtype, case["seed_a"])
    B = workloads.uniform(n, dtype, case["seed_b"])
    ref = B.copy()
    assert oracle.transpose(perm, size, case["alpha"], A, case["beta"], ref) == 0
    dA, pa = to_device(A)
    dB, pb = to_device(B)
    stream = ttx.current_stream()
    z = case["beta"] == 0
    # (a) per call: the generic kernel with the table's configuration
    plan = ttx.ttx_plan_create(code, perm, size)
    try:
        assert ttx.ttx_plan_describe(plan)["config_from_table"][int(z)], "case missing from the shipped table"
    finally:
        ttx.ttx_plan_destroy(plan)
    ttx.ttx_transpose(code, len(perm), perm, size, None, None, case["alpha"], pa, case["beta"], pb, stream)
    assert_parity(from_device(dB), ref, exact=False, what="generic " + case["name"])
    # (b) the plan with its size-specialised kernel, as the throughput step runs it
    dB.copy_(torch.from_numpy(B))
    plan = ttx.ttx_plan_create(code, perm, size)
    try:
        assert ttx.ttx_plan_specialise(plan, z)
        kernel = ttx.ttx_plan_kernel_name(plan, case["beta"], pa, pb)
        assert kernel.startswith("ttx_jit_"), kernel
        _say("  %s" % kernel)
        ttx.ttx_plan_execute(plan, case["alpha"], pa, case["beta"], pb, stream)
    finally:
        ttx.ttx_plan_destroy(plan)
    assert_parity(from_device(dB), ref, exact=False, what="specialised " + case["name"])
    del dA, dB


@pytest.mark.parametrize("dtype,perm", [(F32, (3, 2, 1, 0)), (F32, (2, 0, 3, 1)),
                                        (F64, (1, 0, 3, 2)), (F64, (0, 2, 1, 3))])
def test_literal_160_4d_sampled(dtype, perm):
    """(160,160,160,160): 2.4 GiB (FP32) / 4.9 GiB (FP64) per tensor, checked on
    200K sampled elements computed one by one by the oracle."""
    import torch
    size = workloads.LITERAL_4D
    _say("literal 160^4 %s %s" % (dtype, perm))
    n = _elems(size)
    A = workloads.uniform(n, dtype, 77)
    B = workloads.uniform(n, dtype, 78)
    idx = np.random.default_rng(79).integers(0, n, size=200000)
    idx = np.concatenate([idx, [0, n - 1]])
    expect, off = oracle.sample(perm, size, 1.3, A, 0.7, B, idx)
    got = gpu_transpose(perm, size, 1.3, A, 0.7, B)
    del A, B
    assert_parity(got[off], expect, exact=False)
    torch.cuda.empty_cache()


# -- multiple leading dimensions (BLAS-3 packing) and awkward extents --------------------
@pytest.mark.parametrize("case", workloads.LD_CASES, ids=lambda c: c["name"])
@pytest.mark.parametrize("alpha,beta", workloads.LD_SCALARS)
def test_leading_dimension_cases(case, alpha, beta):
    _say("ld case %s %s %s" % (case["name"], alpha, beta))
    got, ref, exact = _case(case["perm"], case["size"], case["dtype"], alpha, beta,
                            case["outer_a"], case["outer_b"], seed=5)
    # the whole outer B buffer is compared: elements outside the sub-tensor
    # must keep their (random) initial values
    assert_parity(got, ref, exact, case["name"])


def test_fig2_packing_into_contiguous_b():
    got, ref, exact = _case((2, 1, 0), (8, 16, 16), F32, 1.0, 0.0, outer_a=(32, 32, 32), seed=6)
    assert_parity(got, ref, True)


# -- degenerate and edge cases ------------------------------------------------------------
EDGE = [
    ((0,), (1,), None, None),
    ((0,), (1000,), None, None),
    ((0,), (37,), (50,), None),
    ((1, 0), (1, 1), None, None),
    ((0, 1, 2), (3, 4, 5), None, None),                     # identity: flat
    ((0, 1, 2), (3, 4, 5), (4, 4, 5), (3, 6, 5)),           # identity with gaps: preserved
    ((1, 0), (7, 1), None, None),
    ((2, 0, 1, 3), (5, 1, 6, 1), None, None),
    ((1, 0, 2), (1, 7, 5), (3, 7, 5), (7, 2, 5)),           # dropped leading index with ld
    ((1, 0), (1, 1000), None, None),
    ((1, 0), (3, 1000), None, None),
    ((1, 0), (1000, 3), None, None),
    ((1, 0), (65, 63), None, None),
    ((1, 0), (4096, 5), None, None),
    ((2, 1, 0), (129, 3, 130), None, None),
    ((0, 2, 1), (2, 300, 301), None, None),
    ((0, 2, 1), (1000, 3, 4), None, None),
    (tuple(reversed(range(16))), (2, 3, 1, 2, 2, 1, 3, 2, 1, 2, 2, 1, 2, 3, 1, 2), None, None),
    # short stride-1 extents: index groups on the moved side, staged tiles on the kept side
    ((3, 2, 1, 0), (5, 3, 7, 9), None, None),
    ((5, 4, 3, 2, 1, 0), (7, 5, 3, 6, 5, 3), None, None),
    ((2, 3, 0, 1), (3, 11, 7, 13), None, None),
    ((0, 3, 2, 1), (6, 5, 7, 3), None, None),
    ((0, 2, 1), (3, 50, 70), None, None),
    ((0, 5, 1, 4, 2, 3), (24, 5, 4, 3, 17, 3), None, None),
    ((3, 2, 1, 0), (5, 3, 7, 9), (6, 3, 8, 9), (10, 7, 3, 5)),   # gaps block the groups
    ((0, 3, 2, 1), (6, 5, 7, 3), (6, 6, 7, 3), None),
    (tuple(range(1, 16)) + (0,), (3,) + (2,) * 15, None, None),
]


@pytest.mark.parametrize("perm,size,oa,ob", EDGE)
@pytest.mark.parametrize("dtype", [F32, F64])
@pytest.mark.parametrize("alpha,beta", [(1.0, 0.0), (-0.5, 1.0)])
def test_edge_shapes(perm, size, oa, ob, dtype, alpha, beta):
    got, ref, exact = _case(perm, size, dtype, alpha, beta, oa, ob, seed=7)
    assert_parity(got, ref, exact, (perm, size))


@pytest.mark.parametrize("pad_a,pad_b", [(1, 0), (0, 1), (1, 3)])
@pytest.mark.parametrize("dtype", [F32, F64])
def test_misaligned_pointers_take_scalar_paths(pad_a, pad_b, dtype):
    for perm, size in [((2, 1, 0), (64, 9, 48)), ((0, 2, 1), (64, 9, 48)), ((0, 1), (64, 9))]:
        got, ref, exact = _case(perm, size, dtype, 1.25, 0.5, seed=8, pad_a=pad_a, pad_b=pad_b)
        assert_parity(got, ref, exact, (perm, size, pad_a, pad_b))


def test_empty_is_noop():
    B = np.arange(10, dtype=np.float32)
    got = gpu_transpose((1, 0), (0, 10), 1.0, np.zeros(1, dtype=np.float32), 0.0, B)
    assert np.array_equal(got, np.arange(10, dtype=np.float32))


@pytest.mark.parametrize("dtype", [F32, F64])
def test_beta_zero_does_not_read_b(dtype):
    for perm, size in [((2, 1, 0), (33, 5, 70)), ((0, 2, 1), (40, 5, 7)), ((0,), (999,))]:
        got, ref, _ = _case(perm, size, dtype, 2.0, 0.0, seed=9, B_fill=np.nan)
        assert not np.isnan(got).any()
        assert_parity(got, ref, exact=False)
        got, ref, _ = _case(perm, size, dtype, 2.0, -0.0, seed=9, B_fill=np.inf)
        assert np.isfinite(got).all()


@pytest.mark.parametrize("dtype,p", [(F32, 12), (F64, 27)])
def test_contraction_detector(dtype, p):
    """alpha = a = 1 + 2^-p, beta = -1, b = 1 + 2^-(p-1): the unfused result is 0
    exactly; a fused multiply-add would leave 2^-2p."""
    alpha = 1.0 + 2.0 ** -p
    for perm, size in [((1, 0), (64, 64)), ((0, 2, 1), (64, 4, 4)), ((0,), (4096,))]:
        n = _elems(size)
        A = np.full(n, alpha, dtype=dtype)
        B = np.full(n, 1.0 + 2.0 ** -(p - 1), dtype=dtype)
        got = gpu_transpose(perm, size, alpha, A, -1.0, B)
        assert (got == 0).all(), (perm, np.unique(got))


@pytest.mark.parametrize("dtype", [F32, F64])
def test_special_values_pass_through(dtype):
    fi = np.finfo(dtype)
    vals = np.array([0.0, -0.0, np.inf, -np.inf, fi.max, -fi.max, fi.tiny, fi.smallest_subnormal,
                     -fi.smallest_subnormal, 1.0, -1.0, np.nan, 3 * fi.smallest_subnormal],
                    dtype=dtype)
    A = np.resize(vals, 64 * 48).astype(dtype)
    for perm, size in [((1, 0), (64, 48)), ((0, 1), (64, 48)), ((0, 2, 1), (16, 4, 48))]:
        B = np.zeros_like(A)
        ref = B.copy()
        oracle.transpose(perm, size, 1.0, A, 0.0, ref)
        got = gpu_transpose(perm, size, 1.0, A, 0.0, B)
        assert_parity(got, ref, True)   # includes subnormals and signed zeros


@pytest.mark.parametrize("dtype", [F32, F64])
def test_round_trip_on_gpu(dtype):
    perm, size = (2, 0, 3, 1), (37, 70, 19, 23)
    inv = [0] * 4
    for k, p in enumerate(perm):
        inv[p] = k
    A = workloads.uniform(_elems(size), dtype, 10)
    T = gpu_transpose(perm, size, 1.0, A, 0.0, np.zeros_like(A))
    back = gpu_transpose(inv, [size[p] for p in perm], 1.0, T, 0.0, np.zeros_like(A))
    assert_parity(back, A, True)


def test_split_b_in_b_out():
    import torch
    perm, size = (1, 2, 0), (40, 30, 20)
    n = _elems(size)
    A = workloads.uniform(n, F64, 11)
    Bin = workloads.uniform(n, F64, 12)
    ref = Bin.copy()
    oracle.transpose(perm, size, 0.75, A, -1.25, ref)
    dA = torch.from_numpy(A).cuda()
    dBin = torch.from_numpy(Bin).cuda()
    dBout = torch.zeros(n, dtype=torch.float64, device="cuda")
    plan = ttx.ttx_plan_create(ttx.F64, perm, size)
    try:
        ttx.ttx_plan_execute_split(plan, 0.75, dA.data_ptr(), -1.25, dBin.data_ptr(),
                                   dBout.data_ptr(), ttx.current_stream())
    finally:
        ttx.ttx_plan_destroy(plan)
    torch.cuda.synchronize()
    assert_parity(dBout.cpu().numpy(), ref, False)
    assert np.array_equal(dBin.cpu().numpy(), Bin)


# -- every tuner candidate computes the same bits ----------------------------------------
@pytest.mark.parametrize("dtype", [F32, F64])
@pytest.mark.parametrize("perm,size", [((2, 0, 3, 1), (37, 70, 19, 23)), ((0, 2, 1, 3), (40, 9, 11, 13)),
                                       ((1, 0), (7, 3000)), ((1, 0), (300, 5))])
def test_every_candidate_bit_identical(perm, size, dtype):
    cands, _ = ttx.ttx_tune_candidates(ttx.F32 if dtype == F32 else ttx.F64, perm, size,
                                       max_candidates=-1, cap=200000)
    rng = np.random.default_rng(13)
    pick = list(range(min(40, len(cands))))
    pick += list(rng.choice(len(cands), size=min(60, len(cands)), replace=False))
    shapes_seen = set()
    for i in sorted(set(int(k) for k in pick)):
        shapes_seen.add((cands[i].tile_a, cands[i].tile_b))
    # make sure every tile shape of the menu appears at least once
    for c in cands:
        if (c.tile_a, c.tile_b) not in shapes_seen:
            shapes_seen.add((c.tile_a, c.tile_b))
            pick.append(cands.index(c))
    n = _elems(size)
    A = workloads.uniform(n, dtype, 14)
    B = workloads.uniform(n, dtype, 15)
    for beta in (0.7, 0.0):
        ref = B.copy()
        oracle.transpose(perm, size, 1.3, A, beta, ref)
        for i in sorted(set(int(k) for k in pick)):
            got = gpu_transpose(perm, size, 1.3, A, beta, B, plan_config=cands[i])
            assert_parity(got, ref, exact=True, what=str(cands[i].as_dict()))


# -- every workgroup shape (threads per workgroup, LDS row padding) computes the same bits --
def _kind(c):
    if c.flags & ttx.CFG_DENSE:
        return "dense-wide" if c.flags & ttx.CFG_WIDE else "dense"
    if c.family == ttx.FAMILY_PRESERVED and (c.group_a > 1 or c.group_b > 1):
        return "staged"
    return "menu"


@pytest.mark.parametrize("code,perm,size", [
    (ttx.F32, (2, 0, 3, 1), (37, 70, 19, 23)), (ttx.F64, (2, 0, 3, 1), (37, 70, 19, 23)),
    (ttx.F64, (0, 2, 1, 3), (40, 9, 11, 13)), (ttx.F32, (0, 5, 1, 4, 2, 3), (20, 7, 4, 3, 5, 6)),
    (ttx.F32, (1, 0), (7, 3000)), (ttx.C64, (2, 1, 0), (33, 40, 27))])
def test_every_workgroup_variant_bit_identical(code, perm, size):
    """The best-ranked candidate of each tile kind (menu, staged, dense) in
    its workgroup variants (ttx_tune_variants) along each knob: every thread
    count (64..512) at LDS row padding 1, and every padding (0..4) at 256
    threads, each run as a size-specialised kernel compiled for it, gives
    the oracle's bits at beta = 0.7; the 64- and 512-thread variants also at
    beta = 0.  (The knobs are independent template constants of one tile
    code; their cross product is left to the tuner's own runs.)"""
    from gpu_util import TYPES_OF_CODE
    da, db = TYPES_OF_CODE[code]
    cands, _ = ttx.ttx_tune_candidates(code, perm, size, max_candidates=-1, cap=200000)
    bases = {}
    for c in cands:
        bases.setdefault(_kind(c), c)
    n = _elems(size)
    A = workloads.uniform(n, da, 24)
    B = workloads.uniform(n, db, 25)
    refs = {}
    for beta in (0.7, 0.0):
        refs[beta] = B.copy()
        assert oracle.transpose(perm, size, 1.3, A, beta, refs[beta]) == 0
    ran = 0
    for kind, base in sorted(bases.items()):
        variants = ttx.ttx_tune_variants(code, perm, size, base)
        assert len(variants) >= 2 or base.family == ttx.FAMILY_FLAT, kind
        variants = [v for v in variants if v.lds_pad == 1 or v.threads == 256]
        print("%s: %d variants of %s" % (kind, len(variants), base.as_dict()), flush=True)
        for v in variants:
            for beta in ((0.7, 0.0) if v.threads in (64, 512) else (0.7,)):
                got = gpu_transpose(perm, size, 1.3, A, beta, B, plan_config=v)
                assert_parity(got, refs[beta], exact=True, what="%s beta=%g" % (v.as_dict(), beta))
                ran += 1
    assert ran >= 4


@pytest.mark.parametrize("code,perm,size", [
    (ttx.F32, (5, 4, 3, 2, 1, 0), (7, 9, 5, 4, 3, 5)), (ttx.F64, (5, 4, 3, 2, 1, 0), (7, 9, 5, 4, 3, 5)),
    (ttx.F32, (2, 0, 3, 1), (37, 70, 19, 23)), (ttx.F32, (1, 0), (7, 3000)), (ttx.F64, (1, 0), (300, 5)),
    (ttx.F32, (1, 0, 2), (1001, 33, 3)), (ttx.C64, (2, 1, 0), (33, 40, 27)), (ttx.F64_F32, (3, 2, 1, 0), (5, 3, 70, 9)),
    (ttx.F32_F64, (1, 2, 0), (129, 17, 31))])
def test_line_aligned_a_runs_bit_identical(code, perm, size):
    """TTX_CFG_ALIGN_A (tile ranges along A's run start on 128-byte lines):
    the four best-ranked moved tile shapes over a contiguous A run, and its 64- and
    512-thread variants, with the flag set gives the oracle's bits at both
    beta classes, also with misaligned pointers."""
    from gpu_util import TYPES_OF_CODE
    da, db = TYPES_OF_CODE[code]
    cands, _ = ttx.ttx_tune_candidates(code, perm, size, max_candidates=-1, cap=200000)
    seen, picks = set(), []
    for c in cands:
        if c.family != ttx.FAMILY_MOVED or c.flags & ttx.CFG_DENSE:
            continue
        key = (c.tile_a, c.tile_b, c.group_a, c.group_b)
        if key in seen:
            continue
        seen.add(key)
        al = ttx.Config.from_buffer_copy(c)
        al.flags |= ttx.CFG_ALIGN_A
        try:
            variants = ttx.ttx_tune_variants(code, perm, size, al)
        except ttx.TTXError:
            continue   # A's run is not contiguous for these groups
        picks += [v for v in variants if v.threads in (64, 256, 512) and v.lds_pad == 1]
        if len(seen) >= 4:   # the 4 best-ranked moved tile shapes (each config is compiled)
            break
    assert picks, "no candidate takes line-aligned A runs"
    n = _elems(size)
    A = workloads.uniform(n, da, 26)
    B = workloads.uniform(n, db, 27)
    for beta in (0.7, 0.0):
        ref = B.copy()
        assert oracle.transpose(perm, size, 1.3, A, beta, ref) == 0
        for k, v in enumerate(picks):
            pad = (k % 3, (k + 1) % 2)   # element offsets of A and B in their buffers
            _say("  aligned %s beta=%g pad=%s" % (v.as_dict(), beta, pad))
            got = gpu_transpose(perm, size, 1.3, A, beta, B, pad_a=pad[0], pad_b=pad[1], plan_config=v)
            assert_parity(got, ref, exact=True, what="%s beta=%g pad=%s" % (v.as_dict(), beta, pad))


def test_tuner_second_stage_times_workgroup_variants():
    """ttx_tune times the workgroup variants of its fastest candidates after
    the ranked list; whatever wins, the plan that takes it computes the
    oracle's bits."""
    perm, size = (3, 2, 1, 0), (40, 36, 24, 30)
    ttx.ttx_tune_table_clear()
    try:
        best, n = ttx.ttx_tune(ttx.F32, perm, size, beta_is_zero=False, max_candidates=4, reps=2)
        assert n > 4, n
        plan = ttx.ttx_plan_create(ttx.F32, perm, size)
        try:
            info = ttx.ttx_plan_describe(plan)
            assert info["config_from_table"][0] == 1 and info["config"][0] == best.as_dict()
        finally:
            ttx.ttx_plan_destroy(plan)
        n_el = _elems(size)
        A = workloads.uniform(n_el, F32, 31)
        B = workloads.uniform(n_el, F32, 32)
        ref = B.copy()
        assert oracle.transpose(perm, size, 1.3, A, 0.7, ref) == 0
        assert_parity(gpu_transpose(perm, size, 1.3, A, 0.7, B), ref, exact=True, what=str(best.as_dict()))
    finally:
        ttx.ttx_tune_table_clear()


# -- nontemporal and plain stores (separate kernel instances) compute the same bits ---------
@pytest.mark.parametrize("code,perm,size", [
    (ttx.F32, (2, 0, 3, 1), (37, 70, 19, 23)), (ttx.F64, (0, 2, 1, 3), (40, 9, 11, 13)),
    (ttx.F64, (0, 5, 1, 4, 2, 3), (20, 7, 4, 3, 5, 6)), (ttx.F32, (0, 5, 1, 4, 2, 3), (24, 7, 4, 3, 5, 6)),
    (ttx.F32, (1, 0, 2), (3, 4, 700)), (ttx.F64, (0, 1), (64, 9)), (ttx.C64, (2, 1, 0), (33, 40, 27)),
    (ttx.F64_F32, (3, 2, 1, 0), (5, 3, 70, 9))])
def test_store_kinds_bit_identical(code, perm, size):
    """Every tile kind of a problem with TTX_CFG_NT_STORE on and off: the
    generic kernels exist once per store kind and must agree bit for bit."""
    from gpu_util import TYPES_OF_CODE
    da, db = TYPES_OF_CODE[code]
    cands, _ = ttx.ttx_tune_candidates(code, perm, size, max_candidates=-1, cap=200000)
    seen, pick = set(), []
    for c in cands:
        key = (c.tile_a, c.tile_b, c.group_a, c.group_b, c.tile_c, c.flags & (ttx.CFG_DENSE | ttx.CFG_WIDE))
        if key not in seen:
            seen.add(key)
            pick.append(c)
    n = _elems(size)
    A = workloads.uniform(n, da, 16)
    B = workloads.uniform(n, db, 17)
    cx = db in (np.complex64, np.complex128)
    for beta in ((0.5 - 0.25j, 0j) if cx else (0.7, 0.0)):
        alpha = (1.25 + 0.5j) if cx else 1.3
        ref = B.copy()
        oracle.transpose(perm, size, alpha, A, beta, ref)
        for c in pick:
            for nt in (0, ttx.CFG_NT_STORE):
                c.flags = (c.flags & ~ttx.CFG_NT_STORE) | nt
                got = gpu_transpose(perm, size, alpha, A, beta, B, plan_config=c)
                assert_parity(got, ref, exact=True, what=str(c.as_dict()))


# -- dense tiles (run-time extents, rows packed without padding) ----------------------------
DENSE_CASES = [
    ((0, 2, 1), (2, 17835, 2), None, None),            # kept stride-1 index, rows of 2
    ((0, 2, 1, 3), (5, 40, 30, 3), None, None),        # rows of 5
    ((0, 3, 1, 2), (20, 16, 7, 9), None, None),        # rows of 20
    ((1, 0), (7, 3000), None, None),                   # moved, short stride-1 index
    ((2, 0, 1), (6, 7, 500), None, None),
    ((5, 4, 3, 2, 1, 0), (5, 7, 6, 4, 3, 5), None, None),
    ((0, 2, 1), (6, 50, 40), (8, 52, 41), (7, 41, 51)),   # outer sizes on both sides
    ((2, 1, 0), (33, 17, 29), (35, 17, 30), None),
    ((1, 0, 2), (3, 4, 5000), None, None),             # many tiny planes: several per tile
    ((1, 0, 2, 3), (5, 3, 7, 40), None, None),
    ((1, 0, 5, 2, 4, 3), (2, 6, 5, 9, 2, 4), None, None),
    ((1, 0, 2), (3, 4, 700), (4, 5, 700), (5, 3, 701)),  # planes with gaps between them
]


@pytest.mark.parametrize("perm,size,oa,ob", DENSE_CASES)
@pytest.mark.parametrize("dtype", [F32, F64])
def test_dense_tiles(perm, size, oa, ob, dtype):
    code = ttx.F32 if dtype == F32 else ttx.F64
    cands, _ = ttx.ttx_tune_candidates(code, perm, size, outer_a=oa, outer_b=ob, max_candidates=-1,
                                       cap=200000)
    dense = [c for c in cands if c.flags & ttx.CFG_DENSE]
    assert dense, "no dense candidate"
    # every distinct dense shape (first loop order of each), plus a spread of the rest
    seen, pick = set(), []
    for c in dense:
        key = (c.tile_a, c.tile_b, c.group_a, c.group_b, c.tile_c)
        if key not in seen:
            seen.add(key)
            pick.append(c)
    pick += dense[::max(1, len(dense) // 8)]
    # the padded-row staged tiles of the same layouts (kept stride-1 index)
    staged = [c for c in cands if c.family == ttx.FAMILY_PRESERVED and c.group_a > 1
              and not c.flags & ttx.CFG_DENSE]
    pick += staged[::max(1, len(staged) // 6)]
    _say("dense %s %s: %d configs" % (perm, size, len(pick)))
    for alpha, beta in ((1.0, 0.0), (-0.5, 1.0)):
        for i, c in enumerate(pick):
            got, ref, exact = _case(perm, size, dtype, alpha, beta, oa, ob, seed=40 + i % 3, plan_config=c)
            assert_parity(got, ref, exact=exact, what=str(c.as_dict()))


# -- dense tiles over whole units of kept rows (TTX_CFG_WIDE) ----------------------------------
WIDE_CASES = [
    ((0, 3, 1, 2), (20, 16, 7, 9), None, None),          # rows of 5 (FP32) / 10 (FP64) units
    ((0, 5, 1, 4, 2, 3), (24, 5, 4, 3, 7, 3), None, None),
    ((0, 2, 1, 3), (6, 40, 30, 3), None, None),           # FP32: 8-byte units
    ((0, 2, 1), (8, 50, 40), (8, 52, 41), (8, 41, 51)),   # outer sizes on both sides
    ((0, 2, 1, 3), (12, 33, 7, 5), (12, 34, 8, 5), None),
]


@pytest.mark.parametrize("perm,size,oa,ob", WIDE_CASES)
@pytest.mark.parametrize("dtype", [F32, F64])
def test_wide_unit_dense_tiles(perm, size, oa, ob, dtype):
    code = ttx.F32 if dtype == F32 else ttx.F64
    cands, _ = ttx.ttx_tune_candidates(code, perm, size, outer_a=oa, outer_b=ob, max_candidates=-1,
                                       cap=200000)
    wide = [c for c in cands if c.flags & ttx.CFG_WIDE]
    assert wide, "no whole-unit candidate"
    seen, pick = set(), []
    for c in wide:
        key = (c.tile_a, c.tile_b, c.group_a, c.group_b, c.tile_c)
        if key not in seen:
            seen.add(key)
            pick.append(c)
    pick = pick[:24] + wide[::max(1, len(wide) // 6)]
    _say("wide %s %s %s: %d configs" % (perm, size, dtype, len(pick)))
    for alpha, beta in ((1.0, 0.0), (-0.5, 1.0), (1.3, 0.7)):
        for i, c in enumerate(pick):
            got, ref, exact = _case(perm, size, dtype, alpha, beta, oa, ob, seed=50 + i % 3, plan_config=c)
            assert_parity(got, ref, exact=exact, what=str(c.as_dict()))
    # pointers aligned to the element but not to the unit run an element-wise config
    for pad_a, pad_b in ((1, 0), (0, 1), (2, 2)):
        got, ref, exact = _case(perm, size, dtype, 1.25, 0.5, oa, ob, seed=60, pad_a=pad_a, pad_b=pad_b,
                                plan_config=pick[0])
        assert_parity(got, ref, exact, (pad_a, pad_b))


def test_tune_db_appends_each_result(tmp_path):
    """A tuning result is appended to the attached database and is found by
    a new process that attaches the same file."""
    import os
    import subprocess
    db = str(tmp_path / "db.txt")
    ttx.ttx_tune_table_clear()
    ttx.ttx_tune_db_attach(db)
    try:
        best, n = ttx.ttx_tune(ttx.F32, (2, 0, 1), (64, 48, 40), max_candidates=8, reps=2)
        assert n >= 8   # the 8 candidates, then workgroup variants of the fastest
        lines = [l for l in open(db) if not l.startswith("#")]
        assert len(lines) == 1 and lines[0].startswith("d0:b0:")
    finally:
        ttx.ttx_tune_db_detach()
        ttx.ttx_tune_table_clear()
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = ("import sys; sys.path.insert(0, %r); import paper_1607_01249_amd as t; "
            "p = t.ttx_plan_create(0, (2, 0, 1), (64, 48, 40)); "
            "print(t.ttx_plan_describe(p)['config_from_table'][0])" % root)
    r = subprocess.run([sys.executable, "-c", code], env=dict(os.environ, TTX_TUNE_DB=db),
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.split() == ["1"], r.stderr


# -- the bandwidth-ceiling kernels (one pass over the array) ---------------------------------
@pytest.mark.parametrize("n", [1, 7, 4096, 1000003])
def test_ceiling_kernels(n):
    import torch
    src = torch.arange(n * 4, dtype=torch.int32, device="cuda")
    dst = torch.zeros_like(src)
    ttx.ttx_copy_kernel(src.data_ptr(), dst.data_ptr(), n * 16, ttx.current_stream())
    torch.cuda.synchronize()
    assert torch.equal(src, dst)
    for dtype, code in ((F32, ttx.F32), (F64, ttx.F64)):
        x = workloads.uniform(n, dtype, 31)
        y = workloads.uniform(n, dtype, 32)
        # unfused: both products and the sum rounded separately
        want = (dtype.type(1.25) * x) + (dtype.type(-0.5) * y)
        dx, dy = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
        ttx.ttx_axpby_kernel(code, n, 1.25, dx.data_ptr(), -0.5, dy.data_ptr(), ttx.current_stream())
        torch.cuda.synchronize()
        assert np.array_equal(dy.cpu().numpy().view(np.uint8), want.view(np.uint8)), (n, dtype)


# -- grouped tile order (TTX_CFG_GROUPED): a permutation of the tile ids, the same bits ------
@pytest.mark.parametrize("code,perm,size", [
    (ttx.F32, (2, 0, 3, 1), (37, 70, 19, 23)), (ttx.F64, (1, 0), (300, 517)), (ttx.F32, (3, 2, 1, 0), (70, 9, 33, 21)),
    (ttx.F64, (0, 2, 1, 3), (40, 9, 11, 13)), (ttx.F64, (0, 5, 1, 4, 2, 3), (20, 7, 4, 3, 5, 6)),
    (ttx.F32, (0, 5, 1, 4, 2, 3), (24, 7, 4, 3, 5, 6)), (ttx.C64, (2, 1, 0), (33, 40, 27))])
def test_grouped_order_bit_identical(code, perm, size):
    from gpu_util import TYPES_OF_CODE
    da, db = TYPES_OF_CODE[code]
    cands, _ = ttx.ttx_tune_candidates(code, perm, size, max_candidates=-1, cap=200000)
    seen, pick = set(), []
    for c in cands:
        key = (c.tile_a, c.tile_b, c.group_a, c.group_b, c.tile_c, c.flags & (ttx.CFG_DENSE | ttx.CFG_WIDE))
        if key not in seen:
            seen.add(key)
            pick.append(c)
    n = _elems(size)
    A = workloads.uniform(n, da, 18)
    B = workloads.uniform(n, db, 19)
    cx = db in (np.complex64, np.complex128)
    for beta in ((0.5 - 0.25j, 0j) if cx else (0.7, 0.0)):
        alpha = (1.25 + 0.5j) if cx else 1.3
        ref = B.copy()
        oracle.transpose(perm, size, alpha, A, beta, ref)
        specialised = {}
        for c in pick:
            c.flags |= ttx.CFG_GROUPED
            got = gpu_transpose(perm, size, alpha, A, beta, B, plan_config=c)
            assert_parity(got, ref, exact=True, what=str(c.as_dict()))
            # size-specialised too for the two best-ranked tiles of each kind (each one is compiled)
            if specialised.get(_kind(c), 0) < 2:
                specialised[_kind(c)] = specialised.get(_kind(c), 0) + 1
                got = gpu_transpose(perm, size, alpha, A, beta, B, plan_config=c, specialise=True)
                assert_parity(got, ref, exact=True, what="specialised " + str(c.as_dict()))
