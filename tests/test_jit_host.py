"""Host-side checks of the size-specialised kernels (Sec. 2.1): the source the
library generates names the tile of the generic kernel it replaces, and it
compiles with hipRTC for gfx950 without a GPU, with no scratch memory."""
import ctypes
import os
import re
import shutil
import subprocess

import pytest

import paper_1607_01249_amd as ttx

CSRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1607_01249_amd", "csrc")
HEADERS = ["device_types.h", "tile_kernels.h"]
OPTIONS = ["-O3", "-std=c++17", "-ffp-contract=off", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "--offload-arch=gfx950"]

CASES = [  # dtype, perm, size, beta_is_zero
    (ttx.F64, (2, 0, 3, 1), (160, 160, 32, 32), False),
    (ttx.F32, (3, 2, 1, 0), (160, 160, 64, 32), True),
    (ttx.F32, (0, 5, 1, 4, 2, 3), (24, 21, 20, 18, 17, 17), True),
    (ttx.F64, (0, 5, 1, 4, 2, 3), (20, 16, 16, 20, 16, 16), False),
    (ttx.F64, (0, 3, 2, 4, 1), (44, 32, 24, 32, 24), False),
    (ttx.C32, (2, 0, 1), (40, 30, 20), False),
    (ttx.C64, (0, 2, 1), (5, 40, 33), True),
    (ttx.F32_F64, (1, 0, 2), (3, 4, 700), False),
    (ttx.C64_C32, (4, 3, 2, 1, 0), (13, 17, 11, 9, 7), True),
]
IDS = ["d_moved", "s_moved", "s_6d", "d_6d", "d_preserved", "c", "z", "sd", "zc"]


def _source(dtype, perm, size, bz):
    plan = ttx.ttx_plan_create(dtype, perm, size)
    try:
        src = ttx.ttx_plan_specialised_source(plan, bz)
        name = ttx.ttx_plan_kernel_name(plan, 0.0 if bz else 1.0, 1 << 20, 3 << 20)
    finally:
        ttx.ttx_plan_destroy(plan)
    return src, name


def _expected_tile(name):
    """The tile type a generic kernel name runs: k_moved<T, B0, TA, TB, VA, VB, NT>
    runs MovedTile<T, B0, TA, TB, VA, VB, S> (k_<kind>_x<T, S, ...> when the
    types differ; the specialised kernel takes the store kind NT from its
    constant flags), and likewise for the other kinds."""
    m = re.fullmatch(r"k_(moved|preserved|staged|dense)(_x)?<(.*)>", name)
    assert m, name
    args = [a.strip() for a in m.group(3).split(",")]
    t = args[0]
    s, rest = (args[1], args[2:-1]) if m.group(2) else (t, args[1:-1])
    tile = {"moved": "MovedTile", "preserved": "PreservedTile", "staged": "StagedTile", "dense": "DenseTile"}
    # then the store kind (-1: from the constant flags), the workgroup size
    # and, for tiles staged through LDS rows, the row padding
    wg = {"moved": "256, 1, 0", "staged": "256, 1", "preserved": "256", "dense": "256"}[m.group(1)]
    return "ttx::%s<%s, %s, %s, -1, %s>" % (tile[m.group(1)], t, ", ".join(rest), s, wg)


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_source_runs_the_generic_kernels_tile(case):
    src, name = _source(*case)
    assert _expected_tile(name) in src, (name, src[-400:])
    assert 'extern "C" __global__' in src and re.search(r"void ttx_jit_\w+_[0-9a-f]{8}\(", src)
    assert "__builtin_bit_cast(ttx::TileArgsHost, kImage)" in src


def test_nothing_to_specialise_for_flat_and_empty():
    for perm, size in [((0, 1), (64, 9)), ((0,), (1000,)), ((1, 0), (1, 0))]:
        plan = ttx.ttx_plan_create(ttx.F32, perm, size)
        try:
            with pytest.raises(ttx.TTXError):
                ttx.ttx_plan_specialised_source(plan, False)
            assert not ttx.ttx_plan_specialise(plan, False)   # no GPU call: nothing to compile
            assert not ttx.ttx_plan_specialise(plan, True, reps=3)
            assert ttx.ttx_plan_describe(plan)["specialised"] == [0, 0]
        finally:
            ttx.ttx_plan_destroy(plan)


def test_specialised_source_null_and_small_buffer():
    plan = ttx.ttx_plan_create(ttx.F64, (2, 0, 1), (40, 30, 20))
    try:
        buf = ctypes.create_string_buffer(64)
        assert ttx.lib().ttx_plan_specialised_source(plan, 0, buf, 64) == ttx.EINVAL
        assert ttx.lib().ttx_plan_specialised_source(None, 0, buf, 64) == ttx.EINVAL
        assert ttx.lib().ttx_plan_specialise(None, 0, 0, None) == ttx.EINVAL
        assert ttx.lib().ttx_set_auto_specialise(-1) == ttx.EINVAL
        assert ttx.lib().ttx_transpose_cache_info(None, None) == ttx.OK
        perm = (ctypes.c_int * 3)(2, 0, 1)
        size = (ctypes.c_int64 * 3)(40, 30, 20)
        assert ttx.lib().ttx_tune_specialised(ttx.F64, 3, perm, size, None, None, 0, 4, 1, None, None) == ttx.EINVAL
    finally:
        ttx.ttx_plan_destroy(plan)


def _hiprtc():
    for path in ("/opt/rocm/lib/libhiprtc.so", "libhiprtc.so"):
        try:
            return ctypes.CDLL(path)
        except OSError:
            continue
    pytest.skip("hipRTC not installed")


def _compile(src):
    rtc = _hiprtc()
    names = [h.encode() for h in HEADERS]
    texts = [open(os.path.join(CSRC, h), "rb").read() for h in HEADERS]
    prog = ctypes.c_void_p()
    arr = ctypes.c_char_p * len(HEADERS)
    assert rtc.hiprtcCreateProgram(ctypes.byref(prog), src.encode(), b"t.hip", len(HEADERS), arr(*texts),
                                   arr(*names)) == 0
    opts = (ctypes.c_char_p * len(OPTIONS))(*[o.encode() for o in OPTIONS])
    r = rtc.hiprtcCompileProgram(prog, len(OPTIONS), opts)
    n = ctypes.c_size_t()
    rtc.hiprtcGetProgramLogSize(prog, ctypes.byref(n))
    log = ctypes.create_string_buffer(n.value + 1)
    rtc.hiprtcGetProgramLog(prog, log)
    code = b""
    if r == 0:
        rtc.hiprtcGetCodeSize(prog, ctypes.byref(n))
        buf = ctypes.create_string_buffer(n.value)
        rtc.hiprtcGetCode(prog, buf)
        code = buf.raw
    rtc.hiprtcDestroyProgram(ctypes.byref(prog))
    return r, log.value.decode(errors="replace"), code


@pytest.mark.parametrize("case", [CASES[i] for i in (0, 2, 3, 4, 8)], ids=[IDS[i] for i in (0, 2, 3, 4, 8)])
def test_source_compiles_without_scratch(case, tmp_path):
    src, _ = _source(*case)
    r, log, code = _compile(src)
    assert r == 0 and code, log[:3000]
    readobj = shutil.which("llvm-readobj") or "/opt/rocm/llvm/bin/llvm-readobj"
    if not os.path.exists(readobj):
        pytest.skip("llvm-readobj not installed")
    co = tmp_path / "k.co"
    co.write_bytes(code)
    notes = subprocess.run([readobj, "--notes", str(co)], capture_output=True, text=True, check=True).stdout
    assert re.search(r"\.name:\s+ttx_jit_\w+", notes), notes
    # every index constant folded: no private (scratch) memory
    assert re.search(r"\.private_segment_fixed_size:\s+0\b", notes), notes


# -- workgroup variants: threads per workgroup and LDS row padding -----------------------
def _variants(dtype, perm, size, bz):
    plan = ttx.ttx_plan_create(dtype, perm, size)
    try:
        base = ttx.ttx_plan_describe(plan)["config_raw"][1 if bz else 0]
    finally:
        ttx.ttx_plan_destroy(plan)
    return base, ttx.ttx_tune_variants(dtype, perm, size, base)


def test_variants_of_a_moved_tile_span_threads_and_padding():
    base, vs = _variants(ttx.F32, (3, 2, 1, 0), (160, 160, 64, 32), True)
    assert vs[0].as_dict() == base.as_dict()
    seen = {(v.threads, v.lds_pad, v.flags & ttx.CFG_ALIGN_A) for v in vs}
    assert len(seen) == len(vs), "each combination once"
    assert {t for t, _, _ in seen} <= {64, 128, 256, 512} and {p for _, p, _ in seen} <= set(range(5))
    # the pre-compiled shape and at least one other size and padding are there,
    # with line-aligned A runs both ways (A's run is contiguous here)
    assert (256, 1, 0) in seen and len({t for t, _, _ in seen}) >= 3 and len({p for _, p, _ in seen}) == 5
    assert {a for _, _, a in seen} == {0, ttx.CFG_ALIGN_A}
    for v in vs:   # nothing but the workgroup shape and the alignment flag changes
        d, b = v.as_dict(), base.as_dict()
        for k in ("threads", "lds_pad"):
            d.pop(k), b.pop(k)
        d["flags"] &= ~ttx.CFG_ALIGN_A
        b["flags"] &= ~ttx.CFG_ALIGN_A
        assert d == b


def test_variants_of_unpadded_tiles_change_threads_only():
    # direct preserved rows do not pass through LDS: padding is not a dimension
    base, vs = _variants(ttx.F64, (0, 2, 1, 3), (160, 160, 32, 32), False)
    assert base.family == ttx.FAMILY_PRESERVED and (base.group_a, base.group_b) == (1, 1)
    assert len({v.lds_pad for v in vs}) == 1 and len(vs) == len({v.threads for v in vs}) >= 2
    # flat problems run the fixed flat kernel
    base, vs = _variants(ttx.F32, (0, 1), (64, 9), False)
    assert len(vs) == 1


def test_variant_configs_are_checked():
    plan = ttx.ttx_plan_create(ttx.F32, (1, 0), (256, 256))
    try:
        c = ttx.ttx_plan_describe(plan)["config_raw"][0]
        for threads, pad in [(100, 1), (256, 5), (256, -1), (1024, 1)]:
            bad = ttx.Config.from_buffer_copy(c)
            bad.threads, bad.lds_pad = threads, pad
            with pytest.raises(ttx.TTXError):
                ttx.ttx_plan_set_config(plan, False, bad)
        ok = ttx.Config.from_buffer_copy(c)
        ok.threads, ok.lds_pad = 128, 3
        ttx.ttx_plan_set_config(plan, False, ok)
        name = ttx.ttx_plan_kernel_name(plan, 1.0, 1 << 20, 3 << 20)
        assert name.startswith("ttx_jit_moved_float_b_") and "_t128_p3_" in name, name
        src = ttx.ttx_plan_specialised_source(plan, False)
        assert "__launch_bounds__(128)" in src and ", -1, 128, 3, 0>" in src
    finally:
        ttx.ttx_plan_destroy(plan)
    flat = ttx.ttx_plan_create(ttx.F32, (0, 1), (64, 9))
    try:
        c = ttx.Config.from_buffer_copy(ttx.ttx_plan_describe(flat)["config_raw"][0])
        c.threads = 128
        with pytest.raises(ttx.TTXError):
            ttx.ttx_plan_set_config(flat, False, c)
    finally:
        ttx.ttx_plan_destroy(flat)


@pytest.mark.parametrize("threads,pad", [(64, 0), (128, 2), (512, 4)])
def test_variant_sources_compile_without_scratch(threads, pad):
    for dtype, perm, size in [(ttx.F64, (2, 0, 3, 1), (160, 160, 32, 32)),
                              (ttx.F32, (0, 5, 1, 4, 2, 3), (24, 21, 20, 18, 17, 17))]:
        base, vs = _variants(dtype, perm, size, False)
        pick = [v for v in vs if v.threads == threads and (v.lds_pad == pad or base.family != ttx.FAMILY_MOVED)]
        if not pick:
            continue
        plan = ttx.ttx_plan_create(dtype, perm, size)
        try:
            ttx.ttx_plan_set_config(plan, False, pick[0])
            src = ttx.ttx_plan_specialised_source(plan, False)
        finally:
            ttx.ttx_plan_destroy(plan)
        assert "__launch_bounds__(%d)" % threads in src
        r, log, code = _compile(src)
        assert r == 0 and code, log[:3000]


# -- larger moved tiles that exist only as run-time compiled kernels ------------------------
def test_large_tile_shapes_are_listed_apart_from_the_menu():
    for code in (ttx.F32, ttx.F64, ttx.C32, ttx.C64, ttx.F32_F64):
        menu = set(ttx.ttx_tile_shapes(code, ttx.FAMILY_MOVED))
        large = ttx.ttx_tile_shapes(code, ttx.FAMILY_MOVED, run_time_only=True)
        assert menu and large and not menu & set(large), code
        assert ttx.ttx_tile_shapes(code, ttx.FAMILY_PRESERVED, run_time_only=True) == []
    with pytest.raises(ttx.TTXError):
        ttx.ttx_tile_shapes(ttx.F32, ttx.FAMILY_FLAT)


def _large_config(dtype, perm, size, shape, threads=256, align=False):
    plan = ttx.ttx_plan_create(dtype, perm, size)
    c = ttx.Config.from_buffer_copy(ttx.ttx_plan_describe(plan)["config_raw"][0])
    c.tile_a, c.tile_b, c.threads, c.lds_pad = shape[0], shape[1], threads, 1
    c.flags = (c.flags & ~(ttx.CFG_DENSE | ttx.CFG_WIDE | ttx.CFG_ALIGN_A)) | (ttx.CFG_ALIGN_A if align else 0)
    return plan, c


@pytest.mark.parametrize("dtype,perm,size", [(ttx.F32, (3, 2, 1, 0), (160, 160, 64, 32)),
                                             (ttx.F64, (1, 0, 2), (300, 200, 3)),
                                             (ttx.C64, (2, 1, 0), (70, 9, 66))])
def test_large_tiles_run_only_as_specialised_kernels(dtype, perm, size):
    """Each large shape is a valid config of a moved problem; even at the
    pre-compiled workgroup shape (256 threads, padding 1) its kernel is the
    run-time compiled one, and its source compiles with no scratch memory."""
    for k, shape in enumerate(ttx.ttx_tile_shapes(dtype, ttx.FAMILY_MOVED, run_time_only=True)):
        plan, c = _large_config(dtype, perm, size, shape, threads=(256, 512)[k % 2], align=k % 2 == 1)
        try:
            ttx.ttx_plan_set_config(plan, False, c)
            name = ttx.ttx_plan_kernel_name(plan, 1.0, 1 << 20, 3 << 20)
            assert name.startswith("ttx_jit_moved_") and "_%dx%d" % shape in name, name
            src = ttx.ttx_plan_specialised_source(plan, False)
        finally:
            ttx.ttx_plan_destroy(plan)
        if k < 2:   # two compilations per type
            r, log, code = _compile(src)
            assert r == 0 and code, log[:3000]


def test_large_tiles_rejected_outside_the_moved_family():
    plan = ttx.ttx_plan_create(ttx.F64, (0, 2, 1, 3), (160, 160, 32, 32))   # preserved
    try:
        c = ttx.Config.from_buffer_copy(ttx.ttx_plan_describe(plan)["config_raw"][0])
        pres = set(ttx.ttx_tile_shapes(ttx.F64, ttx.FAMILY_PRESERVED))
        c.tile_a, c.tile_b = next(s for s in ttx.ttx_tile_shapes(ttx.F64, ttx.FAMILY_MOVED, run_time_only=True)
                                  if s not in pres)
        with pytest.raises(ttx.TTXError):
            ttx.ttx_plan_set_config(plan, False, c)
    finally:
        ttx.ttx_plan_destroy(plan)


# -- pipelined persistent grids (TTX_CFG_PIPELINED) -------------------------------------------
@pytest.mark.parametrize("dtype,perm,size,kind", [(ttx.F32, (3, 2, 1, 0), (160, 160, 64, 32), "moved"),
                                                  (ttx.F64, (0, 2, 1, 3), (160, 160, 32, 32), "preserved"),
                                                  (ttx.F32, (0, 5, 1, 4, 2, 3), (24, 21, 20, 18, 17, 17),
                                                   None)])
def test_pipelined_configs_run_specialised_and_pipe(dtype, perm, size, kind):
    plan = ttx.ttx_plan_create(dtype, perm, size)
    try:
        c = ttx.Config.from_buffer_copy(ttx.ttx_plan_describe(plan)["config_raw"][0])
        if c.flags & ttx.CFG_DENSE:   # dense tiles always pipeline: the flag is refused
            c.flags |= ttx.CFG_PIPELINED
            with pytest.raises(ttx.TTXError):
                ttx.ttx_plan_set_config(plan, False, c)
            return
        assert kind is None or ttx.FAMILY_NAMES[c.family] == kind
        c.flags |= ttx.CFG_PIPELINED
        ttx.ttx_plan_set_config(plan, False, c)
        name = ttx.ttx_plan_kernel_name(plan, 1.0, 1 << 20, 3 << 20)
        assert name.startswith("ttx_jit_") and "_pl_" in name, name
        src = ttx.ttx_plan_specialised_source(plan, False)
        assert ", true, kHost," in src, src[-400:]
    finally:
        ttx.ttx_plan_destroy(plan)
    r, log, code = _compile(src)
    assert r == 0 and code, log[:3000]


def test_pipelined_flag_refused_for_flat_problems():
    plan = ttx.ttx_plan_create(ttx.F32, (0, 1), (64, 9))
    try:
        c = ttx.Config.from_buffer_copy(ttx.ttx_plan_describe(plan)["config_raw"][0])
        c.flags |= ttx.CFG_PIPELINED
        with pytest.raises(ttx.TTXError):
            ttx.ttx_plan_set_config(plan, False, c)
    finally:
        ttx.ttx_plan_destroy(plan)
