"""Host-side checks of the C ABI (no GPU): exported symbols, argument
validation against the oracle's, the planner's index merging and family
choice on the paper's examples, merge invariance through the oracle, and
the candidate ranking of the tuner."""
import itertools
import json
import os
import re
import subprocess

import numpy as np
import pytest

import oracle
import paper_1607_01249_amd as ttx

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLDEN = os.path.join(ROOT, "tests", "golden")


def _golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def _declared_symbols():
    text = open(os.path.join(ROOT, "include", "ttx.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ttx_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    names = _declared_symbols()
    assert "ttx_transpose" in names and len(names) >= 15
    L = ttx.lib()
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    out = subprocess.run(["nm", "-D", "--defined-only", ttx._ttx.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (ttx_\w+)", out))
    assert set(names) <= exported, set(names) - exported


def test_binding_wraps_every_declared_symbol():
    for n in _declared_symbols():
        if n in ("ttx_status_string", "ttx_last_error", "ttx_version"):
            continue
        assert hasattr(ttx._ttx, n), n


def test_status_strings():
    L = ttx.lib()
    for s in range(9):
        assert L.ttx_status_string(s)
    assert b"ttx" in L.ttx_version()


# -- validation: the library's synchronous checks agree with the oracle's -------------
INVALID = [
    dict(dtype=8, perm=(0, 1), size=(2, 3)),
    dict(dtype=0, perm=(0, 0), size=(2, 3)),
    dict(dtype=0, perm=(0, 2), size=(2, 3)),
    dict(dtype=0, perm=(1, 0), size=(2, -1)),
    dict(dtype=0, perm=(1, 0), size=(2, 3), outer_a=(1, 3)),
    dict(dtype=0, perm=(1, 0), size=(2, 3), outer_b=(3, 1)),
    dict(dtype=1, perm=(2, 1, 0), size=(4, 5, 6), outer_a=(4, 5, 5)),
    dict(dtype=0, perm=tuple(range(17)), size=(1,) * 17),
]


@pytest.mark.parametrize("case", INVALID)
def test_plan_validation_matches_oracle(case):
    expect = oracle.check(case["dtype"], case["perm"], case["size"], case.get("outer_a"),
                          case.get("outer_b"))
    assert expect != oracle.OK
    with pytest.raises(ttx.TTXError) as err:
        ttx.ttx_plan_create(case["dtype"], case["perm"], case["size"], case.get("outer_a"),
                            case.get("outer_b"))
    assert err.value.status == expect


def test_transpose_rejects_overlap_and_null_without_gpu():
    # validation happens before any HIP call, so these work without a GPU
    base = 1 << 40
    with pytest.raises(ttx.TTXError) as err:
        ttx.ttx_transpose(0, 2, (1, 0), (2, 3), None, None, 1.0, base, 0.0, base + 20)
    assert err.value.status == ttx.EOVERLAP
    with pytest.raises(ttx.TTXError) as err:
        ttx.ttx_transpose(0, 2, (1, 0), (2, 3), None, None, 1.0, None, 0.0, base)
    assert err.value.status == ttx.EINVAL
    with pytest.raises(ttx.TTXError) as err:   # misaligned for FP64
        ttx.ttx_transpose(1, 2, (1, 0), (2, 3), None, None, 1.0, base + 4, 0.0, base + 4096)
    assert err.value.status == ttx.EINVAL
    # an empty tensor is a no-op even with dangling pointers
    ttx.ttx_transpose(0, 2, (1, 0), (0, 3), None, None, 1.0, None, 0.0, None)


# -- planner on the paper's examples ------------------------------------------------------
def _describe(dtype, perm, size, outer_a=None, outer_b=None):
    p = ttx.ttx_plan_create(dtype, perm, size, outer_a, outer_b)
    try:
        return ttx.ttx_plan_describe(p)
    finally:
        ttx.ttx_plan_destroy(p)


def test_sec21_merge_example():
    g = _golden("sec21_merge_example.json")
    d = _describe(0, g["perm"], g["size"])
    assert d["perm"] == g["merged_perm"] and d["size"] == g["merged_size"]
    assert d["family"] == "moved"


def test_fig2_packing_no_merge():
    g = _golden("fig2_packing.json")
    d = _describe(0, g["perm"], g["size"], g["outer_a"], g["outer_b"])
    assert d["perm"] == g["merged_perm"] and d["size"] == g["merged_size"]
    assert d["family"] == g["family"]
    assert d["stride_a"] == g["stride_a"]
    # stride_b is reported per A index: A index m sits at B position perm^-1(m)
    inv = [g["perm"].index(m) for m in range(3)]
    assert d["stride_b"] == [g["stride_b"][inv[m]] for m in range(3)]


def test_stride1_kept_examples_are_preserved():
    for case in _golden("stride1_kept_examples.json")["cases"]:
        d = _describe(1, case["perm"], case["size"])
        assert d["family"] == case["family"], case
        assert d["perm"] == case["merged_perm"] and d["size"] == case["merged_size"]


def test_ld_blocks_merge_and_contiguous_merges():
    # outer_b[2] = 50 != 48 keeps i2 and i3 apart; contiguous B merges them
    d = _describe(1, (1, 0, 2, 3), (384, 96, 48, 32), (400, 100, 48, 32), (100, 400, 50, 32))
    assert d["n"] == 4 and d["family"] == "moved"
    d = _describe(1, (1, 0, 2, 3), (384, 96, 48, 32), (400, 100, 48, 32), None)
    assert d["perm"] == [1, 0, 2] and d["size"] == [384, 96, 48 * 32]
    d = _describe(1, (1, 0, 2, 3), (384, 96, 48, 32))
    assert d["perm"] == [1, 0, 2] and d["size"] == [384, 96, 48 * 32]


def test_awkward_and_size1():
    d = _describe(0, (1, 2, 3, 0), (7, 1023, 33, 65))
    assert d["perm"] == [1, 0] and d["size"] == [7, 1023 * 33 * 65]
    d = _describe(0, (2, 0, 1, 3), (5, 1, 6, 1))
    assert d["perm"] == [1, 0] and d["size"] == [5, 6]
    d = _describe(0, (1, 0), (1, 1))
    assert d["family"] == "flat" and d["elements"] == 1
    d = _describe(0, (0, 1, 2), (3, 4, 5))
    assert d["family"] == "flat" and d["size"] == [60]
    d = _describe(0, (0, 1), (3, 4), (5, 4))
    assert d["family"] == "preserved" and d["size"] == [3, 4]
    d = _describe(0, (1, 0), (3, 0))
    assert d["family"] == "empty"
    # a dropped leading index with a leading dimension leaves a strided index 0
    d = _describe(0, (1, 0, 2), (1, 7, 5), (3, 7, 5))
    assert d["stride_a"][0] == 3


def _canonical_outer(d):
    """The planner's merged problem as (perm, size, outer_a, outer_b).  A
    leading extent-1 index carries the strides of merged index 0 when they
    are not 1 (extent-1 indices with leading dimensions were dropped)."""
    n, perm, size, sa, sb = d["n"], d["perm"], d["size"], d["stride_a"], d["stride_b"]
    outer_a = [sa[0]] + [sa[m + 1] // sa[m] for m in range(n - 1)] + [size[-1]]
    outer_b = [sb[perm[0]]] + [sb[perm[k + 1]] // sb[perm[k]] for k in range(n - 1)] + [size[perm[-1]]]
    return [0] + [p + 1 for p in perm], [1] + list(size), outer_a, outer_b


def test_merge_invariance_through_oracle():
    """The oracle on the original problem equals the oracle on the planner's
    merged, size-1-free problem, on the same buffers (A and B unchanged)."""
    rng = np.random.default_rng(5)
    cases = [((1, 2, 0), (3, 4, 5), None, None),
             ((0, 5, 1, 4, 2, 3), (3, 2, 4, 2, 3, 2), None, None),
             ((1, 2, 3, 0), (7, 3, 2, 5), None, None),
             ((2, 3, 0, 1), (2, 3, 4, 5), None, None),
             ((1, 0, 2, 3), (5, 4, 3, 2), (6, 4, 3, 2), (4, 7, 3, 2)),
             ((2, 0, 1, 3), (3, 1, 4, 1), (3, 1, 4, 1), None),
             ((0, 1, 2), (3, 4, 5), (3, 6, 5), None)]
    for perm, size, oa, ob in cases:
        d = _describe(1, perm, size, oa, ob)
        cperm, csize, coa, cob = _canonical_outer(d)
        size_b = [size[p] for p in perm]
        na = int(np.prod(oa or size))
        nb = int(np.prod(ob or size_b))
        A = rng.random(na)
        B0 = rng.random(nb)
        B1, B2 = B0.copy(), B0.copy()
        assert oracle.transpose(perm, size, 1.25, A, -0.5, B1, oa, ob) == 0
        assert oracle.transpose(cperm, csize, 1.25, A, -0.5, B2, coa, cob) == 0
        assert np.array_equal(B1, B2), (perm, size, d)


def test_merge_random_against_oracle():
    rng = np.random.default_rng(6)
    for _ in range(200):
        n = int(rng.integers(1, 7))
        perm = tuple(int(p) for p in rng.permutation(n))
        size = tuple(int(rng.choice([1, 2, 3, 4])) for _ in range(n))
        size_b = [size[p] for p in perm]
        oa = tuple(s + int(rng.integers(0, 2)) for s in size) if rng.random() < 0.5 else None
        ob = tuple(s + int(rng.integers(0, 2)) for s in size_b) if rng.random() < 0.5 else None
        d = _describe(0, perm, size, oa, ob)
        cperm, csize, coa, cob = _canonical_outer(d)
        A = rng.random(int(np.prod(oa or size)), dtype=np.float32)
        B0 = rng.random(int(np.prod(ob or size_b)), dtype=np.float32)
        B1, B2 = B0.copy(), B0.copy()
        oracle.transpose(perm, size, 2.0, A, 0.0, B1, oa, ob)
        oracle.transpose(cperm, csize, 2.0, A, 0.0, B2, coa, cob)
        assert np.array_equal(B1, B2), (perm, size, oa, ob, d)
        # families follow the merged permutation
        fam = "flat" if d["n"] == 1 else ("preserved" if d["perm"][0] == 0 else "moved")
        assert d["family"] == fam


# -- candidate ranking (Sec. 2.1 stages 2-3, Sec. 2.3) ------------------------------------
def test_candidate_list_is_bounded_and_sorted():
    cands, cost = ttx.ttx_tune_candidates(0, (3, 2, 1, 0), (160, 160, 64, 32), cap=4096)
    assert len(cands) == 200  # default capacity
    assert cost == sorted(cost)
    few, few_cost = ttx.ttx_tune_candidates(0, (3, 2, 1, 0), (160, 160, 64, 32), max_candidates=10)
    assert len(few) == 10 and few_cost == sorted(few_cost)
    # each kernel kind keeps a quarter of a bounded list; the rest are the cheapest
    dense = [c for c in cands if c.flags & ttx.CFG_DENSE]
    assert len(dense) >= 50 and len([c for c in few if c.flags & ttx.CFG_DENSE]) >= 2
    assert few_cost[0] == cost[0]
    allc, _ = ttx.ttx_tune_candidates(0, (3, 2, 1, 0), (160, 160, 64, 32), max_candidates=-1, cap=100000)
    # every menu shape x 4 flag sets x the loop orders of each index grouping:
    # 4! orders with single indices, and 3! when B's short stride-1 index (32)
    # is grouped with the next B index (the grid then has 3 indices)
    fixed = [c for c in allc if not c.flags & ttx.CFG_DENSE]
    assert len(fixed) == 22 * 4 * (24 + 6)
    assert {(c.group_a, c.group_b) for c in allc} == {(1, 1), (1, 2)}
    # dense tiles: run-time extents within the capacity, the same loop orders
    dense = [c for c in allc if c.flags & ttx.CFG_DENSE]
    assert dense and len(dense) % (4 * 6) == 0
    for c in dense:
        assert 1 <= c.tile_a and 1 <= c.tile_b and c.tile_a * c.tile_b <= ttx.DENSE_CAP[ttx.F32]
    for c in cands:
        assert sorted(c.order[:c.n_order]) == [0, 1, 2, 3]


def test_dense_tiles_validation_and_choice():
    F = ttx.CFG_DENSE
    # short rows of the kept stride-1 index (n0 = 2): dense tiles hold whole
    # rows, so n0 * tile_a * tile_b is bounded by the capacity
    cands, _ = ttx.ttx_tune_candidates(0, (0, 2, 1), (2, 17835, 2), max_candidates=-1, cap=100000)
    dense = [c for c in cands if c.flags & F]
    assert dense and all(c.group_a >= 2 and c.group_b >= 2 for c in dense)
    assert all(2 * c.tile_a * c.tile_b <= ttx.DENSE_CAP[ttx.F32] for c in dense)
    # the heuristic default picks a dense tile here (padded rows would idle most lanes)
    d = _describe(0, (0, 2, 1), (2, 17835, 2))
    assert d["config"][1]["flags"] & F
    p = ttx.ttx_plan_create(0, (0, 2, 1), (2, 17835, 2))
    try:
        good = ttx.Config.from_buffer_copy(dense[0])
        ttx.ttx_plan_set_config(p, 1, good)
        assert "k_dense<float" in ttx.ttx_plan_kernel_name(p, 1, 1 << 40, 1 << 41)
        bad = ttx.Config.from_buffer_copy(dense[0])
        bad.tile_a, bad.tile_b = 64, 16            # 2 * 64 * 16 > 1024
        with pytest.raises(ttx.TTXError):
            ttx.ttx_plan_set_config(p, 1, bad)
        bad = ttx.Config.from_buffer_copy(dense[0])
        bad.group_a = bad.group_b = 1              # dense preserved tiles need row groups
        with pytest.raises(ttx.TTXError):
            ttx.ttx_plan_set_config(p, 1, bad)
    finally:
        ttx.ttx_plan_destroy(p)
    # moved problems take dense tiles of any extents within the capacity
    cands, _ = ttx.ttx_tune_candidates(1, (1, 0), (7, 3000), max_candidates=-1, cap=100000)
    dense = [c for c in cands if c.flags & F]
    assert dense and {c.tile_a for c in dense} >= {7}
    assert all(c.tile_a * c.tile_b <= ttx.DENSE_CAP[ttx.F64] for c in dense)
    # flat problems have no dense form
    p = ttx.ttx_plan_create(0, (0, 1), (10, 10))
    try:
        cfg = ttx.Config.from_buffer_copy(ttx.ttx_plan_describe(p)["config_raw"][1])
        cfg.flags |= F
        with pytest.raises(ttx.TTXError):
            ttx.ttx_plan_set_config(p, 1, cfg)
    finally:
        ttx.ttx_plan_destroy(p)


def test_blocking_heuristic_prefers_exact_tiles_and_skinny_for_short_index():
    c, _ = ttx.ttx_tune_candidates(0, (1, 0), (7, 100000), max_candidates=1)
    # a 7-long stride-1 index: a dense tile 7 wide, or one of the skinny shapes
    assert (c[0].flags & ttx.CFG_DENSE and c[0].tile_a == 7) or c[0].tile_a in (4, 8)
    # the remainder rule: no partial edge tile -- each extent is a multiple of
    # the tile edge, or one tile spans it whole (B rows then lie back to back)
    c, _ = ttx.ttx_tune_candidates(0, (1, 0), (96, 80), max_candidates=1)
    ta, tb = c[0].tile_a, c[0].tile_b
    assert (96 % ta == 0 or ta >= 96) and (80 % tb == 0 or tb >= 80), (ta, tb)
    c, _ = ttx.ttx_tune_candidates(0, (1, 0), (4096, 4096), max_candidates=1)
    assert c[0].tile_a * c[0].tile_b == 4096     # the largest tiles for a large square transpose


def test_loop_heuristic_prefers_small_strides_fastest():
    # (2,1,0) on (1024, 64, 1024): the middle index has stride 1024 in both
    # tensors while a step of either tile index jumps 64*65536 elements in
    # one of them
    c, cost = ttx.ttx_tune_candidates(0, (2, 1, 0), (1024, 64, 1024), max_candidates=-1, cap=100000)
    # orders that enumerate the middle index among the resident tiles tie; the
    # ones that leave it last (after both tile indices) cost more
    orders = {tuple(x.order[:3]): cc for x, cc in zip(c, cost)
              if (x.tile_a, x.tile_b, x.flags) == (c[0].tile_a, c[0].tile_b, 0)}
    assert orders[(1, 0, 2)] < orders[(0, 2, 1)]


def test_plan_set_config_validation():
    p = ttx.ttx_plan_create(0, (2, 1, 0), (96, 128, 80))
    try:
        d = ttx.ttx_plan_describe(p)
        cfg = d["config_raw"][1]
        ttx.ttx_plan_set_config(p, 1, cfg)
        bad = ttx.Config.from_buffer_copy(cfg)
        bad.tile_a = 17
        with pytest.raises(ttx.TTXError):
            ttx.ttx_plan_set_config(p, 1, bad)
        bad = ttx.Config.from_buffer_copy(cfg)
        bad.order[0] = bad.order[1]
        with pytest.raises(ttx.TTXError):
            ttx.ttx_plan_set_config(p, 1, bad)
        bad = ttx.Config.from_buffer_copy(cfg)
        bad.family = ttx.FAMILY_PRESERVED
        with pytest.raises(ttx.TTXError):
            ttx.ttx_plan_set_config(p, 1, bad)
    finally:
        ttx.ttx_plan_destroy(p)


def test_plan_config_handoff_between_threads():
    """A plan's configuration is replaced as one object: a thread reading it
    while another swaps between two configurations always sees one of the
    two whole, never fields of both."""
    import threading
    perm, size = (2, 0, 3, 1), (70, 33, 19, 23)
    cands, _ = ttx.ttx_tune_candidates(ttx.F32, perm, size, max_candidates=-1, cap=100000)
    a = cands[0]
    b = next(c for c in cands if (c.tile_a, c.tile_b) != (a.tile_a, a.tile_b) and
             list(c.order[:4]) != list(a.order[:4]) and c.flags != a.flags)
    key = lambda d: json.dumps(d, sort_keys=True)
    want = {key(a.as_dict()), key(b.as_dict())}
    p = ttx.ttx_plan_create(ttx.F32, perm, size)
    stop = threading.Event()
    seen, errors = set(), []

    def writer():
        i = 0
        while not stop.is_set():
            ttx.ttx_plan_set_config(p, 0, a if i % 2 == 0 else b)
            i += 1

    def reader():
        for _ in range(20000):
            k = key(ttx.ttx_plan_describe(p)["config"][0])
            seen.add(k)
            if k not in want:
                errors.append(k)
                break

    try:
        ttx.ttx_plan_set_config(p, 0, a)
        w = threading.Thread(target=writer)
        w.start()
        try:
            reader()
        finally:
            stop.set()
            w.join()
    finally:
        ttx.ttx_plan_destroy(p)
    assert not errors, errors[:1]
    assert seen <= want


def test_tune_table_roundtrip(tmp_path):
    ttx.ttx_tune_table_clear()
    path = str(tmp_path / "table.txt")
    with open(path, "w") as f:
        f.write("# comment\n")
        f.write("d0:b1:n3:s96,128,80:p2,1,0:a1,96,12288:o10240,80,1 | 3 32 16 256 1 1 1 3 0 2 1 | 12.5\n")
    ttx.ttx_tune_table_load(path)
    assert ttx.ttx_tune_table_size() == 1
    d = _describe(0, (2, 1, 0), (96, 128, 80))
    assert d["config_from_table"] == [0, 1]
    assert d["config"][1]["tile_a"] == 32 and d["config"][1]["order"] == [0, 2, 1]
    out = str(tmp_path / "saved.txt")
    ttx.ttx_tune_table_save(out)
    assert "s96,128,80" in open(out).read()
    ttx.ttx_tune_table_clear()
    d = _describe(0, (2, 1, 0), (96, 128, 80))
    assert d["config_from_table"] == [0, 0]


def test_tune_table_keeps_workgroup_shape(tmp_path):
    """Entries with another workgroup size and LDS padding (l<pad>) load,
    reach the plan, and are written back the same way; an out-of-range
    padding is a malformed line."""
    ttx.ttx_tune_table_clear()
    path = str(tmp_path / "table.txt")
    line = "d0:b1:n3:s96,128,80:p2,1,0:a1,96,12288:o10240,80,1 | 3 32 16 128 1 1 1 3 0 2 1 l3 | 12.5\n"
    with open(path, "w") as f:
        f.write(line)
    try:
        ttx.ttx_tune_table_load(path)
        d = _describe(0, (2, 1, 0), (96, 128, 80))
        assert d["config_from_table"] == [0, 1]
        assert d["config"][1]["threads"] == 128 and d["config"][1]["lds_pad"] == 3
        out = str(tmp_path / "saved.txt")
        ttx.ttx_tune_table_save(out)
        assert " 128 1 1 1 3 0 2 1 l3 | " in open(out).read()
        with open(path, "w") as f:
            f.write(line.replace(" l3 ", " l9 "))
        with pytest.raises(ttx.TTXError):
            ttx.ttx_tune_table_load(path)
    finally:
        ttx.ttx_tune_table_clear()


def test_fastdiv_host_exhaustive_sample(tmp_path):
    src = tmp_path / "fd.cpp"
    src.write_text(r'''
#include "ttx_internal.h"
#include <cstdio>
#include <random>
int main() {
    std::mt19937_64 rng(7);
    const uint32_t ds[] = {1, 2, 3, 5, 7, 10, 24, 48, 641, 65535, 65536, 1u << 31, 0xffffffffu};
    for (uint32_t d : ds) {
        ttx::FastDiv f(d);
        for (int i = 0; i < 200000; ++i) {
            uint32_t n = i < 1000 ? uint32_t(i) : (i < 2000 ? 0xffffffffu - uint32_t(i) : uint32_t(rng()));
            if (f.div(n) != n / d) { std::printf("bad %u %u\n", n, d); return 1; }
        }
    }
    for (int i = 0; i < 200000; ++i) {
        uint32_t d = uint32_t(rng()) % 100000 + 1, n = uint32_t(rng());
        ttx::FastDiv f(d);
        if (f.div(n) != n / d) { std::printf("bad %u %u\n", n, d); return 1; }
    }
    return 0;
}
''')
    exe = tmp_path / "fd"
    subprocess.run(["g++", "-O2", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                    "-I" + os.path.join(ROOT, "paper_1607_01249_amd", "csrc"), str(src), "-o", str(exe)],
                   check=True)
    subprocess.run([str(exe)], check=True)


# -- complex element types (c and z) ------------------------------------------------------
COMPLEX_SHAPES = [((2, 0, 3, 1), (37, 70, 19, 23)), ((0, 2, 1), (5, 40, 33)), ((1, 0), (7, 3000)),
                  ((1, 0, 2), (3, 4, 700)), ((0,), (100,)), ((0, 2, 1), (64, 9, 48))]


@pytest.mark.parametrize("code", [ttx.C32, ttx.C64])
@pytest.mark.parametrize("perm,size", COMPLEX_SHAPES)
def test_complex_plans_and_candidates(code, perm, size):
    tname = "ttx::cf32" if code == ttx.C32 else "ttx::cf64"
    plan = ttx.ttx_plan_create(code, perm, size)
    try:
        info = ttx.ttx_plan_describe(plan)
        assert info["dtype"] == code
        name = ttx.ttx_plan_kernel_name(plan, 1, 1 << 40, 1 << 41)
        assert tname in name, name
        if code == ttx.C64:   # one element is a whole 16-byte access: no vector variants
            assert not any(v in name for v in (", 2>", ", 2, 2>", ", 2, 1>", ", 1, 2>")), name
    finally:
        ttx.ttx_plan_destroy(plan)
    cands, cost = ttx.ttx_tune_candidates(code, perm, size, max_candidates=-1, cap=200000)
    assert cands and cost == sorted(cost)
    n0 = size[0] if perm[0] == 0 else 1
    for c in cands:
        if c.flags & ttx.CFG_DENSE:
            rows = n0 if c.family == ttx.FAMILY_PRESERVED else 1
            assert rows * c.tile_a * c.tile_b * max(1, c.tile_c) <= ttx.DENSE_CAP[code]


def test_complex_c32_uses_the_fp64_menu_shapes():
    """Single complex elements have the FP64 byte size: same tile menu."""
    perm, size = (2, 0, 3, 1), (37, 70, 19, 23)
    shapes = {}
    for code in (ttx.F64, ttx.C32, ttx.C64):
        cands, _ = ttx.ttx_tune_candidates(code, perm, size, max_candidates=-1, cap=200000)
        shapes[code] = {(c.tile_a, c.tile_b) for c in cands if not c.flags & ttx.CFG_DENSE}
    assert shapes[ttx.C32] == shapes[ttx.F64]
    assert shapes[ttx.C64] != shapes[ttx.F64] and (32, 32) in shapes[ttx.C64]


def test_complex_argument_errors_need_no_gpu():
    perm, size = (1, 0), (4, 5)
    # complex scalars for a real element type
    with pytest.raises(ttx.TTXError) as e:
        ttx.ttx_transpose_c(ttx.F32, 2, perm, size, None, None, 1 + 1j, 1 << 40, 0.0, 1 << 41)
    assert e.value.status == ttx.EINVAL
    with pytest.raises(ttx.TTXError) as e:
        ttx.ttx_transpose_c(ttx.F64, 2, perm, size, None, None, 1.0, 1 << 40, 2j, 1 << 41)
    assert e.value.status == ttx.EINVAL
    # element alignment: 8 bytes for single complex, 16 for double complex
    with pytest.raises(ttx.TTXError) as e:
        ttx.ttx_transpose_c(ttx.C32, 2, perm, size, None, None, 1j, (1 << 40) + 4, 0.0, 1 << 41)
    assert e.value.status == ttx.EINVAL
    with pytest.raises(ttx.TTXError) as e:
        ttx.ttx_transpose_c(ttx.C64, 2, perm, size, None, None, 1j, (1 << 40) + 8, 0.0, 1 << 41)
    assert e.value.status == ttx.EINVAL
    # overlap uses the complex element size (20 elements of 16 bytes)
    with pytest.raises(ttx.TTXError) as e:
        ttx.ttx_transpose_c(ttx.C64, 2, perm, size, None, None, 1j, 1 << 40, 0.0, (1 << 40) + 304)
    assert e.value.status == ttx.EOVERLAP
    # oracle and library agree on the dtype codes
    for code in (ttx.C32, ttx.C64):
        assert oracle.check(code, perm, size) == oracle.OK
    assert oracle.check(8, perm, size) != oracle.OK


# -- mixed precision (sd, ds, cz, zc) ---------------------------------------------------------
MIXED = [(ttx.F32_F64, ttx.F64, "double, float"), (ttx.F64_F32, ttx.F32, "float, double"),
         (ttx.C32_C64, ttx.C64, "ttx::cf64, ttx::cf32"), (ttx.C64_C32, ttx.C32, "ttx::cf32, ttx::cf64")]


@pytest.mark.parametrize("code,b_type,names", MIXED)
@pytest.mark.parametrize("perm,size", COMPLEX_SHAPES)
def test_mixed_plans_use_b_type_menus(code, b_type, names, perm, size):
    plan = ttx.ttx_plan_create(code, perm, size)
    try:
        info = ttx.ttx_plan_describe(plan)
        assert info["dtype"] == code
        name = ttx.ttx_plan_kernel_name(plan, 1, 1 << 40, 1 << 41)
        assert "_x<" + names + "," in name, name
    finally:
        ttx.ttx_plan_destroy(plan)
    got, _ = ttx.ttx_tune_candidates(code, perm, size, max_candidates=-1, cap=200000)
    same, _ = ttx.ttx_tune_candidates(b_type, perm, size, max_candidates=-1, cap=200000)
    shape = lambda c: (c.family, c.tile_a, c.tile_b, c.group_a, c.group_b, c.tile_c, c.flags & ttx.CFG_DENSE)
    assert {shape(c) for c in got} == {shape(c) for c in same}


def test_mixed_argument_errors_need_no_gpu():
    perm, size = (1, 0), (4, 5)   # 20 elements
    big = 1 << 40
    cases = [(ttx.F32_F64, big, big + 4096 + 4, ttx.EINVAL),    # B (FP64) not 8-byte aligned
             (ttx.F64_F32, big + 4, big + 4096, ttx.EINVAL),    # A (FP64) not 8-byte aligned
             (ttx.C32_C64, big + 8, big + 4096 + 8, ttx.EINVAL),  # B (double complex) needs 16
             (ttx.F32_F64, big, big + 72, ttx.EOVERLAP),        # A spans 80 bytes (FP32)
             (ttx.F64_F32, big, big + 80, ttx.EOVERLAP)]        # A spans 160 bytes (FP64)
    for code, a, b, status in cases:
        with pytest.raises(ttx.TTXError) as e:
            ttx.ttx_transpose(code, 2, perm, size, None, None, 1.0, a, 0.0, b)
        assert e.value.status == status, (code, a, b)
    with pytest.raises(ttx.TTXError) as e:   # complex scalars for a real pair
        ttx.ttx_transpose_c(ttx.F32_F64, 2, perm, size, None, None, 1j, big, 0.0, big + 4096)
    assert e.value.status == ttx.EINVAL
    for a, b in ((0, 1), (1, 0), (2, 3), (3, 2)):
        assert oracle.check(b, perm, size, dtype_a=a) == oracle.OK


@pytest.mark.parametrize("code", [ttx.C32, ttx.C64, ttx.F32_F64, ttx.C64_C32])
def test_batch_plans_complex_and_mixed_problems_per_call(code):
    """The persistent kernel takes FP32/FP64 problems; complex and mixed ones
    get their per-call configs (and no tiles of the persistent kernel)."""
    alpha = 0.5 - 1j if code in (ttx.C32, ttx.C64, ttx.C64_C32) else 1.0
    q = ttx.make_problem(code, (1, 0), (40, 50), alpha, 1 << 40, 0.0, 1 << 41)
    r = ttx.make_problem(ttx.F32, (1, 0), (40, 50), 1.0, 1 << 42, 0.0, 1 << 43)
    cfgs, tiles = ttx.ttx_batch_plan([q, r])
    assert tiles[0] == 0 and tiles[1] > 0
    plan = ttx.ttx_plan_create(code, (1, 0), (40, 50))
    try:
        want = ttx.ttx_plan_describe(plan)["config"][1]
    finally:
        ttx.ttx_plan_destroy(plan)
    assert cfgs[0].as_dict() == want


def test_batch_rejects_complex_scalars_for_real_problems():
    q = ttx.make_problem(ttx.F64, (1, 0), (40, 50), 1j, 1 << 40, 0.0, 1 << 41)
    with pytest.raises(ttx.TTXError) as e:
        ttx.ttx_batch_plan([q])
    assert e.value.status == ttx.EINVAL


# -- GEMM operand packing (host planning) ------------------------------------------------------
def test_pack_describe_splits_whole_and_ragged_panels():
    n, cfgs = ttx.ttx_pack_describe(ttx.F32, ttx.PACK_ROWS, 37, 19, 40, 8)
    assert n == 5 * 8 * 19 and len(cfgs) == 2
    assert cfgs[0].family == ttx.FAMILY_PRESERVED       # panel rows stay contiguous
    n, cfgs = ttx.ttx_pack_describe(ttx.F32, ttx.PACK_ROWS, 32, 19, 40, 8)
    assert n == 32 * 19 and len(cfgs) == 1
    n, cfgs = ttx.ttx_pack_describe(ttx.F64, ttx.PACK_COLS, 19, 37, 20, 8)
    assert n == 19 * 5 * 8 and len(cfgs) == 2
    assert cfgs[0].family == ttx.FAMILY_MOVED
    n, cfgs = ttx.ttx_pack_describe(ttx.C32_C64, ttx.PACK_COLS, 0, 37, 20, 8)
    assert n == 0 and cfgs == []


def test_pack_argument_errors_need_no_gpu():
    big = 1 << 40
    for args, status in [((ttx.F32, 4, 4, 4, 4, 2), ttx.EINVAL),       # unknown kind
                         ((ttx.F32, ttx.PACK_MFMA_A, 4, 4, 4, 12), ttx.EINVAL),   # panel not dividing 64
                         ((ttx.F32, ttx.PACK_MFMA_B, 4, 4, 4, 128), ttx.EINVAL),
                         ((ttx.F32, 0, 4, 4, 3, 2), ttx.EINVAL),       # ld < rows
                         ((ttx.F32, 0, 4, 4, 4, 0), ttx.EINVAL),       # panel < 1
                         ((8, 0, 4, 4, 4, 2), ttx.EINVAL)]:            # unknown dtype
        with pytest.raises(ttx.TTXError) as e:
            ttx.ttx_pack(*args, 1.0, big, big + (1 << 20))
        assert e.value.status == status, args
    with pytest.raises(ttx.TTXError) as e:   # A spans 4*4*4 = 64 bytes, P 64 bytes
        ttx.ttx_pack(ttx.F32, 0, 4, 4, 4, 2, 1.0, big, big + 60)
    assert e.value.status == ttx.EOVERLAP
    with pytest.raises(ttx.TTXError) as e:   # complex scale for real panels
        ttx.ttx_pack(ttx.F32, 0, 4, 4, 4, 2, 1j, big, big + 4096)
    assert e.value.status == ttx.EINVAL


def test_mfma_pack_describe_and_gemm_argument_errors_need_no_gpu():
    """Matrix-core panels hold ceil(extent/panel)*panel*K elements, K = k
    rounded up to whole blocks of 64/panel; the GEMM refuses unsupported
    (dtype, panel) pairs and bad extents before any launch."""
    for kind, rows, cols, panel, want in [(ttx.PACK_MFMA_A, 37, 13, 16, 48 * 16), (ttx.PACK_MFMA_B, 13, 37, 16, 48 * 16),
                                          (ttx.PACK_MFMA_A, 100, 7, 32, 128 * 8), (ttx.PACK_MFMA_A, 64, 8, 16, 64 * 8),
                                          (ttx.PACK_ROWS, 37, 13, 16, 48 * 13)]:
        n, parts = ttx.ttx_pack_describe(ttx.F32, kind, rows, cols, rows, panel)
        assert n == want, (kind, rows, cols, panel)
    big = 1 << 40
    for args in [(ttx.F64, 32, 4, 4, 4), (ttx.C32, 16, 4, 4, 4), (ttx.F32, 8, 4, 4, 4)]:
        with pytest.raises(ttx.TTXError) as e:
            ttx.ttx_gemm_panels(*args, big, big + 4096, big + 8192, 4)
        assert e.value.status == ttx.EUNSUPPORTED, args
    for args in [(ttx.F32, 16, -1, 4, 4, 4), (ttx.F32, 16, 8, 4, 4, 4), (ttx.F32, 16, 4, 4, -2, 4)]:
        with pytest.raises(ttx.TTXError) as e:
            ttx.ttx_gemm_panels(*args[:5], big, big + 4096, big + 8192, args[5])
        assert e.value.status == ttx.EINVAL, args


# -- the tune table as a database shared across processes ------------------------------------
KEY_PLAIN = "d0:b1:n3:s96,128,80:p2,1,0:a1,96,12288:o10240,80,1"


def test_tune_db_keeps_lowest_time_and_creates_missing_files(tmp_path):
    ttx.ttx_tune_table_clear()
    db = str(tmp_path / "db.txt")
    with open(db, "w") as f:
        f.write(KEY_PLAIN + " | 3 32 16 256 1 1 1 3 0 2 1 | 12.5\n")
        f.write(KEY_PLAIN + " | 3 64 32 256 0 1 1 3 2 0 1 | 9.0\n")    # faster, appended later
        f.write(KEY_PLAIN + " | 3 16 16 256 0 1 1 3 1 0 2 | 30.0\n")
    try:
        ttx.ttx_tune_db_attach(db)
        d = _describe(0, (2, 1, 0), (96, 128, 80))
        assert d["config_from_table"] == [0, 1]
        assert d["config"][1]["tile_a"] == 64 and d["config"][1]["order"] == [2, 0, 1]
    finally:
        ttx.ttx_tune_db_detach()
        ttx.ttx_tune_table_clear()
    fresh = str(tmp_path / "new_db.txt")
    try:
        ttx.ttx_tune_db_attach(fresh)
        assert open(fresh).read().startswith("# ttx tune table")
    finally:
        ttx.ttx_tune_db_detach()


def test_tune_db_from_the_environment_in_a_new_process(tmp_path):
    import subprocess
    import sys
    db = str(tmp_path / "env_db.txt")
    with open(db, "w") as f:
        f.write(KEY_PLAIN + " | 3 32 16 256 1 1 1 3 0 2 1 | 12.5\n")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = ("import sys; sys.path.insert(0, %r); import paper_1607_01249_amd as t; "
            "p = t.ttx_plan_create(0, (2, 1, 0), (96, 128, 80)); d = t.ttx_plan_describe(p); "
            "print(d['config_from_table'][1], d['config'][1]['tile_a'])" % root)
    env = dict(os.environ, TTX_TUNE_DB=db)
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    assert r.stdout.split() == ["1", "32"]


def test_tune_table_from_the_environment_is_read_only(tmp_path):
    import subprocess
    import sys
    table = str(tmp_path / "shipped.txt")
    with open(table, "w") as f:
        f.write(KEY_PLAIN + " | 3 32 16 256 1 1 1 3 0 2 1 | 12.5\n")
    before = open(table).read()
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = ("import sys; sys.path.insert(0, %r); import paper_1607_01249_amd as t; "
            "print(t.ttx_tune_table_size()); p = t.ttx_plan_create(0, (2, 1, 0), (96, 128, 80)); "
            "print(t.ttx_plan_describe(p)['config_from_table'][1])" % root)
    r = subprocess.run([sys.executable, "-c", code], env=dict(os.environ, TTX_TUNE_TABLE=table),
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    assert r.stdout.split() == ["1", "1"]
    assert open(table).read() == before


def test_shipped_table_covers_the_large_cases():
    """Every line of the shipped tune table parses and names a config the
    planner accepts: each throughput case's plan (large, complex, mixed)
    takes its generic entry, and the entries for specialised execution
    (prefix j:) name valid configs too."""
    import os
    import numpy as np
    import workloads
    tcode = {np.dtype(np.float32): ttx.F32, np.dtype(np.float64): ttx.F64,
             np.dtype(np.complex64): ttx.C32, np.dtype(np.complex128): ttx.C64}
    cases = [dict(c, code=tcode[np.dtype(c["dtype"])]) for c in workloads.large_cases()]
    cases += [dict(c, code=ttx.CODE_OF[(tcode[np.dtype(c["dtype_a"])], tcode[np.dtype(c["dtype"])])])
              for c in workloads.complex_cases() + workloads.mixed_cases()]
    table = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                         "paper_1607_01249_amd", "tune", "gfx950.txt")
    ttx.ttx_tune_table_clear()
    try:
        ttx.ttx_tune_table_load(table)
        lines = [l for l in open(table) if l.strip() and not l.startswith("#")]
        assert ttx.ttx_tune_table_size() == len(lines)
        spec_keys = {l.split("|")[0].strip()[2:] for l in lines if l.startswith("j:")}
        for c in cases:
            plan = ttx.ttx_plan_create(c["code"], c["perm"], c["size"])
            try:
                info = ttx.ttx_plan_describe(plan)
                z = 1 if c["beta"] == 0 else 0
                assert info["config_from_table"][z] == 1, c["name"]
                key = "d%d:b%d:n%d:s%s:p%s:a%s:o%s" % (
                    info["dtype"], z, info["n"], ",".join(map(str, info["size"])), ",".join(map(str, info["perm"])),
                    ",".join(map(str, info["stride_a"])), ",".join(map(str, info["stride_b"])))
                if key in spec_keys:   # the specialised entry's config must be valid for the plan
                    line = [l for l in lines if l.startswith("j:" + key + " |")][0]
                    f = line.split("|")[1].split()
                    cfg = ttx.Config()
                    cfg.family, cfg.tile_a, cfg.tile_b, cfg.threads, cfg.flags = map(int, f[:5])
                    cfg.group_a, cfg.group_b, cfg.n_order = map(int, f[5:8])
                    for i in range(cfg.n_order):
                        cfg.order[i] = int(f[8 + i])
                    for tok in f[8 + cfg.n_order:]:   # optional c<planes> and l<padding>
                        if tok[0] == "c":
                            cfg.tile_c = int(tok[1:])
                        elif tok[0] == "l":
                            cfg.lds_pad = int(tok[1:])
                    ttx.ttx_plan_set_config(plan, z, cfg)
                    spec_keys.discard(key)
            finally:
                ttx.ttx_plan_destroy(plan)
        assert not spec_keys, spec_keys
    finally:
        ttx.ttx_tune_table_clear()


C_CONSUMER = r"""
#include <stdio.h>
#include <string.h>
#include "ttx.h"
/* A plain C (not C++) consumer of the boundary: host-only entry points. */
int main(void) {
    int perm[3] = {2, 1, 0};
    int64_t size[3] = {96, 128, 80};
    ttx_plan *p = NULL;
    ttx_plan_info info;
    ttx_contraction *c = NULL;
    ttx_contraction_info ci;
    int la[2] = {0, 2}, lb[2] = {2, 1}, lc[2] = {0, 1};
    int64_t sa[2] = {70, 33}, sb[2] = {33, 45}, sc[2] = {70, 45};
    int ta[64], tb[64], count = 0;
    if (ttx_plan_create(&p, TTX_F32, 3, perm, size, NULL, NULL) != TTX_OK) return 1;
    if (ttx_plan_describe(p, &info) != TTX_OK || info.family != TTX_FAMILY_MOVED) return 2;
    ttx_plan_destroy(p);
    perm[0] = 3;   /* not a permutation */
    if (ttx_plan_create(&p, TTX_F32, 3, perm, size, NULL, NULL) != TTX_EPERM) return 3;
    if (strlen(ttx_last_error()) == 0 || strlen(ttx_status_string(TTX_EPERM)) == 0) return 4;
    if (ttx_contraction_create(&c, TTX_F64, 2, la, sa, 2, lb, sb, 2, lc, sc) != TTX_OK) return 5;
    if (ttx_contraction_describe(c, &ci) != TTX_OK || ci.m != 70 || ci.n != 45 || ci.k != 33) return 6;
    ttx_contraction_destroy(c);
    if (ttx_tile_shapes(TTX_F32, TTX_FAMILY_MOVED, 0, ta, tb, 64, &count) != TTX_OK || count < 16) return 7;
    printf("ok %s\n", ttx_version());
    return 0;
}
"""


def test_header_is_a_c_abi(tmp_path):
    """include/ttx.h compiles as C99 with gcc (no C++ in the signatures), and
    a C program linked against libttx.so runs its host-only entry points."""
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    rocm_inc = "/opt/rocm/include"
    if not gcc or not os.path.isdir(rocm_inc):
        pytest.skip("gcc or the ROCm headers are not installed")
    src = tmp_path / "consumer.c"
    src.write_text(C_CONSUMER)
    exe = tmp_path / "consumer"
    libdir = os.path.dirname(ttx.lib()._name)
    subprocess.run([gcc, "-std=c99", "-Wall", "-Wextra", "-Werror", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"),
                    "-I", rocm_inc, str(src), "-L", libdir, "-lttx", "-Wl,-rpath," + libdir, "-o", str(exe)],
                   check=True, capture_output=True, text=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert out.returncode == 0 and out.stdout.startswith("ok "), (out.returncode, out.stdout, out.stderr)
