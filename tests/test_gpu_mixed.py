"""GPU parity for mixed-precision transpositions (Table 1 "sd", "ds", "cz",
"zc": A and B in different precisions), through the C ABI, against the CPU
oracle.

The A element is converted to B's type as it is loaded (widening exact,
narrowing to nearest) and the update is computed in B's type on both sides,
so bit-identity is expected; the bar is at most 1 ulp (bit-exact for
alpha = 1, beta = 0).
"""
import sys

import numpy as np
import pytest

import oracle
import paper_1607_01249_amd as ttx
import workloads
from gpu_util import C32, C64, F32, F64, REAL_OF, assert_parity, dtype_code, gpu_transpose

pytestmark = pytest.mark.gpu

PAIRS = [(F32, F64), (F64, F32), (C32, C64), (C64, C32)]
PAIR_IDS = ["sd", "ds", "cz", "zc"]


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _scalars(db, beta_zero=False):
    if db in (C32, C64):
        return complex(0.75, -1.25), (0j if beta_zero else complex(-0.5, 0.375))
    return 1.3, (0.0 if beta_zero else 0.7)


def _case(perm, size, da, db, alpha, beta, outer_a=None, outer_b=None, seed=0, plan_config=None,
          B_fill=None, pad_a=0, pad_b=0):
    size_b = [size[p] for p in perm]
    A = workloads.uniform(workloads.elements(outer_a or size), da, seed=7000 + seed) * 3
    if B_fill is None:
        B = workloads.uniform(workloads.elements(outer_b or size_b), db, seed=8000 + seed)
    else:
        B = np.full(workloads.elements(outer_b or size_b), B_fill, dtype=db)
    ref = B.copy()
    assert oracle.transpose(perm, size, alpha, A, beta, ref, outer_a, outer_b) == 0
    got = gpu_transpose(perm, size, alpha, A, beta, B, outer_a, outer_b, pad_a, pad_b, plan_config)
    return got, ref, alpha == 1 and beta == 0


REDUCED = {"4d": (37, 70, 19, 23), "5d": (13, 17, 11, 9, 7), "6d": (5, 7, 6, 4, 3, 5)}
REDUCED_CASES = [(rank, perm, pair, bz) for rank in ("4d", "5d", "6d")
                 for perm in workloads.LARGE_PERMS[rank] for pair in range(4) for bz in (False, True)]


@pytest.mark.parametrize("rank,perm,pair,beta_zero", REDUCED_CASES)
def test_reduced_large_perms_mixed(rank, perm, pair, beta_zero):
    da, db = PAIRS[pair]
    alpha, beta = _scalars(db, beta_zero)
    got, ref, exact = _case(perm, REDUCED[rank], da, db, alpha, beta, seed=1)
    assert_parity(got, ref, exact, (rank, perm, PAIR_IDS[pair]))


@pytest.mark.parametrize("pair", range(4), ids=PAIR_IDS)
def test_plain_conversion_exact(pair):
    da, db = PAIRS[pair]
    for perm, size in [((2, 1, 0), (33, 40, 27)), ((0, 2, 1), (24, 9, 31)), ((1, 0), (300, 7)),
                       ((0,), (1001,))]:
        got, ref, exact = _case(perm, size, da, db, 1.0, 0.0, seed=2)
        assert exact
        assert_parity(got, ref, True, (perm, size))


@pytest.mark.parametrize("pair", [1, 3], ids=["ds", "zc"])
def test_narrowing_rounds_to_nearest(pair):
    """Values on and beside float midpoints, subnormal results and overflow."""
    da, db = PAIRS[pair]
    u = 2.0 ** -24
    vals = [1.0 + u, 1.0 + 3 * u, 1.0 + u * (1 + 2.0 ** -20), -(1.0 + 3 * u), 2.0 ** -150,
            3.0 * 2.0 ** -150, 0.1, 1e-40, -7e-46, 3.4e38, 3.5e38]
    parts = np.resize(np.array(vals, dtype=F64), 2 * 64 * 48)
    A = parts[: 64 * 48] if da == F64 else parts.view(C64)[: 64 * 48].copy()
    for perm, size in [((1, 0), (64, 48)), ((0, 1), (64, 48)), ((0, 2, 1), (16, 4, 48))]:
        B = np.zeros(64 * 48, dtype=db)
        ref = B.copy()
        oracle.transpose(perm, size, 1.0, A, 0.0, ref)
        got = gpu_transpose(perm, size, 1.0, A, 0.0, B)
        assert_parity(got, ref, True, perm)


EDGE = [
    ((1, 0), (1, 1), None, None),
    ((0,), (777,), (900,), (1000,)),
    ((2, 0, 1), (3, 1, 200), None, None),
    ((1, 0), (7, 3000), None, None),
    ((0, 2, 1), (2, 300, 70), None, None),
    ((0, 2, 1, 3), (5, 40, 30, 3), None, None),
    ((3, 2, 1, 0), (5, 3, 7, 9), (6, 3, 8, 9), (10, 7, 3, 5)),
    ((0, 2, 1), (6, 50, 40), (8, 52, 41), (7, 41, 51)),
    ((1, 0, 2), (3, 4, 700), (4, 5, 700), (5, 3, 701)),
    ((5, 4, 3, 2, 1, 0), (7, 5, 3, 6, 5, 3), None, None),
]


@pytest.mark.parametrize("perm,size,oa,ob", EDGE)
@pytest.mark.parametrize("pair", range(4), ids=PAIR_IDS)
def test_edge_and_leading_dimension_shapes(perm, size, oa, ob, pair):
    da, db = PAIRS[pair]
    alpha, beta = _scalars(db)
    got, ref, exact = _case(perm, size, da, db, alpha, beta, oa, ob, seed=3)
    assert_parity(got, ref, exact, (perm, size))


@pytest.mark.parametrize("pad_a,pad_b", [(1, 0), (0, 1), (1, 3)])
@pytest.mark.parametrize("pair", [0, 1], ids=["sd", "ds"])
def test_misaligned_pointers_take_scalar_paths(pad_a, pad_b, pair):
    da, db = PAIRS[pair]
    for perm, size in [((2, 1, 0), (64, 9, 48)), ((0, 2, 1), (64, 9, 48)), ((0, 1), (64, 9))]:
        got, ref, exact = _case(perm, size, da, db, 1.25, 0.5, seed=8, pad_a=pad_a, pad_b=pad_b)
        assert_parity(got, ref, exact, (perm, size, pad_a, pad_b))


@pytest.mark.parametrize("pair", range(4), ids=PAIR_IDS)
def test_beta_zero_does_not_read_b(pair):
    da, db = PAIRS[pair]
    nan = np.array([complex(np.nan, np.nan) if db in (C32, C64) else np.nan], dtype=db)[0]
    alpha, beta = _scalars(db, beta_zero=True)
    for perm, size in [((2, 1, 0), (33, 5, 70)), ((0, 2, 1), (40, 5, 7)), ((0,), (999,))]:
        got, ref, _ = _case(perm, size, da, db, alpha, beta, seed=5, B_fill=nan)
        assert not np.isnan(got.view(REAL_OF.get(db, db))).any()
        assert_parity(got, ref, False)


@pytest.mark.parametrize("pair", range(4), ids=PAIR_IDS)
@pytest.mark.parametrize("perm,size", [((2, 0, 3, 1), (37, 70, 19, 23)), ((0, 2, 1, 3), (40, 9, 11, 13)),
                                       ((0, 2, 1), (5, 40, 33)), ((1, 0), (7, 3000)),
                                       ((1, 0, 2), (3, 4, 700)), ((0,), (5000,))])
def test_every_tile_kind_bit_identical(perm, size, pair):
    da, db = PAIRS[pair]
    cands, _ = ttx.ttx_tune_candidates(dtype_code(da, db), perm, size, max_candidates=-1, cap=200000)
    seen, pick = set(), []
    for c in cands:   # one config per distinct tile (kind, shape, groups, planes)
        key = (c.tile_a, c.tile_b, c.group_a, c.group_b, c.tile_c, c.flags & ttx.CFG_DENSE)
        if key not in seen:
            seen.add(key)
            pick.append(c)
    pick += cands[:8]
    _say("mixed candidates %s %s %s: %d configs" % (perm, size, PAIR_IDS[pair], len(pick)))
    n = workloads.elements(size)
    A = workloads.uniform(n, da, 14) * 3
    B = workloads.uniform(n, db, 15)
    for bz in (False, True):
        alpha, beta = _scalars(db, bz)
        ref = B.copy()
        oracle.transpose(perm, size, alpha, A, beta, ref)
        for c in pick:
            got = gpu_transpose(perm, size, alpha, A, beta, B, plan_config=c)
            assert_parity(got, ref, exact=True, what=str(c.as_dict()))


@pytest.mark.parametrize("pair,perm,size", [(0, (3, 2, 1, 0), (160, 160, 64, 32)),
                                            (1, (2, 0, 3, 1), (160, 160, 32, 32)),
                                            (2, (0, 2, 1, 3), (160, 160, 32, 32)),
                                            (3, (3, 2, 1, 0), (160, 160, 32, 16))])
def test_full_size_mixed(pair, perm, size):
    da, db = PAIRS[pair]
    _say("full-size mixed %s %s %s" % (PAIR_IDS[pair], perm, size))
    alpha, beta = _scalars(db)
    got, ref, exact = _case(perm, size, da, db, alpha, beta, seed=30)
    assert_parity(got, ref, exact, (PAIR_IDS[pair], perm))
