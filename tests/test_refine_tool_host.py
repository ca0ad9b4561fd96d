"""Host-side checks of the offline table-refinement tool
(paper_1607_01249_amd/tune/refine_workgroups.py): the variant lists it
times are configs the planner accepts or refuses cleanly, and the table it
writes loads back with its entries (no GPU: the timing itself needs one)."""
import os

import pytest

import paper_1607_01249_amd as ttx
from paper_1607_01249_amd.tune import refine_workgroups as rw

CASES = [(ttx.F32, (3, 2, 1, 0), (160, 160, 64, 32)), (ttx.F64, (0, 2, 1, 3), (160, 160, 32, 32)),
         (ttx.F32, (0, 5, 1, 4, 2, 3), (24, 21, 20, 18, 17, 17))]


def _base(code, perm, size):
    plan = ttx.ttx_plan_create(code, perm, size)
    try:
        return ttx.Config.from_buffer_copy(ttx.ttx_plan_describe(plan)["config_raw"][0])
    finally:
        ttx.ttx_plan_destroy(plan)


def _accepted(code, perm, size, variants):
    ok = 0
    for v in variants:
        plan = ttx.ttx_plan_create(code, perm, size)
        try:
            ttx.ttx_plan_set_config(plan, False, v)
            ok += 1
        except ttx.TTXError:
            pass
        finally:
            ttx.ttx_plan_destroy(plan)
    return ok


@pytest.mark.parametrize("code,perm,size", CASES)
def test_variant_lists_are_planner_configs(code, perm, size):
    base = _base(code, perm, size)
    large = rw.large_variants(ttx, code, perm, size, base)
    pipe = rw.pipelined_variants(ttx, code, perm, size, base)
    shapes = rw.shape_variants(ttx, code, perm, size, base)
    moved = base.family == ttx.FAMILY_MOVED and not base.flags & ttx.CFG_DENSE
    tiled = base.family in (ttx.FAMILY_MOVED, ttx.FAMILY_PRESERVED) and not base.flags & ttx.CFG_DENSE
    assert bool(large) == moved and bool(shapes) == moved and bool(pipe) == tiled
    assert all(v.flags & ttx.CFG_PIPELINED for v in pipe)
    large_shapes = set(ttx.ttx_tile_shapes(code, ttx.FAMILY_MOVED, run_time_only=True))
    assert {(v.tile_a, v.tile_b) for v in large} <= large_shapes
    for vs in (large, pipe, shapes):
        if vs:
            assert _accepted(code, perm, size, vs) >= 1


def test_written_table_loads_back(tmp_path):
    code, perm, size = CASES[0]
    plan = ttx.ttx_plan_create(code, perm, size)
    try:
        info = ttx.ttx_plan_describe(plan)
    finally:
        ttx.ttx_plan_destroy(plan)
    base = ttx.Config.from_buffer_copy(info["config_raw"][0])
    v = rw.pipelined_variants(ttx, code, perm, size, base)[0]
    src = tmp_path / "in.txt"
    src.write_text("")
    dst = tmp_path / "out.txt"
    rw.write_table(str(src), str(dst), {rw.table_key(info, 0): (v, 12.5)})
    line = dst.read_text().strip()
    assert line.startswith("j:") and line.endswith("| 12.500")
    ttx.ttx_tune_table_clear()
    try:
        ttx.ttx_tune_table_load(str(dst))
        assert ttx.ttx_tune_table_size() == 1
        back = tmp_path / "back.txt"
        ttx.ttx_tune_table_save(str(back))
        saved = [l for l in back.read_text().splitlines() if l.startswith("j:")]
        assert len(saved) == 1 and saved[0].split(" | ")[:2] == line.split(" | ")[:2]
    finally:
        ttx.ttx_tune_table_clear()
