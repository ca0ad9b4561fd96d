"""ctypes binding of the ttx C ABI (``include/ttx.h``).

Argument marshalling only: every call goes straight to ``libttx.so``; no
step of the transposition runs in Python.  Functions named ``ttx_*`` mirror
the C entry points one to one (integers, sequences and raw pointers in,
status-checked); ``transpose`` is a convenience wrapper that takes torch
tensors as storage (their data pointers and dtypes are used, their shapes
are not: the column-major interpretation comes from ``size``).

The library must be built (``python -m paper_1607_01249_amd.build`` or
``__graft_entry__.build()``); importing a function that needs it raises
when ``libttx.so`` is missing.  There is no fallback path.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libttx.so")
MAX_DIMS = 16

F32, F64, C32, C64 = 0, 1, 2, 3
# mixed precision (A's type first): sd, ds, cz, zc
F32_F64, F64_F32, C32_C64, C64_C32 = 4, 5, 6, 7
ELEM_BYTES = {F32: 4, F64: 8, C32: 8, C64: 16}
# (A's element type, B's element type) of every data-type code
TYPES_OF = {F32: (F32, F32), F64: (F64, F64), C32: (C32, C32), C64: (C64, C64),
            F32_F64: (F32, F64), F64_F32: (F64, F32), C32_C64: (C32, C64), C64_C32: (C64, C32)}
CODE_OF = {v: k for k, v in TYPES_OF.items()}
OK, EINVAL, EPERM, EOVERLAP, EUNSUPPORTED, ENOMEM, EHIP, EBUSY, ENOTFOUND = range(9)
FAMILY_EMPTY, FAMILY_FLAT, FAMILY_PRESERVED, FAMILY_MOVED = range(4)
FAMILY_NAMES = {0: "empty", 1: "flat", 2: "preserved", 3: "moved"}
CFG_XCD_SWIZZLE, CFG_NT_STORE, CFG_DENSE, CFG_WIDE, CFG_GROUPED, CFG_ALIGN_A, CFG_PIPELINED = 1, 2, 4, 8, 16, 32, 64
PACK_ROWS, PACK_COLS, PACK_MFMA_A, PACK_MFMA_B = 0, 1, 2, 3
DENSE_CAP = {F32: 1024, F64: 1024, C32: 1024, C64: 512}
DENSE_CAP.update({code: DENSE_CAP[b] for code, (a, b) in TYPES_OF.items() if a != b})

i64 = ctypes.c_int64
i64p = ctypes.POINTER(ctypes.c_int64)
ip = ctypes.POINTER(ctypes.c_int)
vp = ctypes.c_void_p


class TTXError(RuntimeError):
    def __init__(self, status, detail):
        self.status = status
        super().__init__("ttx status %d: %s" % (status, detail))


class Config(ctypes.Structure):
    _fields_ = [("family", ctypes.c_int), ("tile_a", ctypes.c_int), ("tile_b", ctypes.c_int),
                ("threads", ctypes.c_int), ("n_order", ctypes.c_int),
                ("order", ctypes.c_int * MAX_DIMS), ("flags", ctypes.c_int),
                ("group_a", ctypes.c_int), ("group_b", ctypes.c_int), ("tile_c", ctypes.c_int),
                ("lds_pad", ctypes.c_int)]

    def __init__(self, *args, **kw):
        # the pre-compiled kernels' workgroup shape unless given
        kw.setdefault("threads", 256)
        kw.setdefault("lds_pad", 1)
        super().__init__(*args, **kw)

    def as_dict(self):
        return dict(family=FAMILY_NAMES[self.family], tile_a=self.tile_a, tile_b=self.tile_b,
                    threads=self.threads, order=list(self.order[:self.n_order]), flags=self.flags,
                    group_a=self.group_a, group_b=self.group_b, tile_c=self.tile_c, lds_pad=self.lds_pad)


class PlanInfo(ctypes.Structure):
    _fields_ = [("dtype", ctypes.c_int), ("family", ctypes.c_int), ("n", ctypes.c_int),
                ("perm", ctypes.c_int * MAX_DIMS), ("size", i64 * MAX_DIMS),
                ("stride_a", i64 * MAX_DIMS), ("stride_b", i64 * MAX_DIMS),
                ("elements", i64), ("extent_a_bytes", i64), ("extent_b_bytes", i64),
                ("config", Config * 2), ("config_from_table", ctypes.c_int * 2),
                ("specialised", ctypes.c_int * 2)]


class Problem(ctypes.Structure):
    _fields_ = [("dtype", ctypes.c_int), ("n", ctypes.c_int), ("perm", ctypes.c_int * MAX_DIMS),
                ("size", i64 * MAX_DIMS), ("outer_a", i64 * MAX_DIMS), ("outer_b", i64 * MAX_DIMS),
                ("has_outer_a", ctypes.c_int), ("has_outer_b", ctypes.c_int),
                ("alpha", ctypes.c_double), ("beta", ctypes.c_double),
                ("A", vp), ("B_in", vp), ("B", vp),
                ("alpha_im", ctypes.c_double), ("beta_im", ctypes.c_double)]


class BatchInfo(ctypes.Structure):
    _fields_ = [("count", ctypes.c_int), ("grid", ctypes.c_int), ("variants_used", ctypes.c_int),
                ("tuned", ctypes.c_int), ("total_tiles", i64), ("algorithmic_bytes", i64), ("chunks", i64),
                ("per_call", ctypes.c_int)]


class ContractionInfo(ctypes.Structure):
    _fields_ = [("m", i64), ("n", i64), ("k", i64), ("panel", ctypes.c_int), ("transposed_a", ctypes.c_int),
                ("transposed_b", ctypes.c_int), ("pack_kind_a", ctypes.c_int), ("pack_kind_b", ctypes.c_int),
                ("n_m", ctypes.c_int), ("n_n", ctypes.c_int), ("n_k", ctypes.c_int),
                ("order_m", ctypes.c_int * MAX_DIMS), ("order_n", ctypes.c_int * MAX_DIMS),
                ("order_k", ctypes.c_int * MAX_DIMS), ("workspace_bytes", i64)]


class Request(ctypes.Structure):
    _fields_ = [("problem", Problem), ("arrival_ns", i64), ("keep_result", ctypes.c_int)]


class ServerOpts(ctypes.Structure):
    _fields_ = [("hbm_fraction", ctypes.c_double), ("arena_bytes", i64), ("slots", ctypes.c_int),
                ("max_batch", ctypes.c_int), ("max_batch_bytes", i64), ("max_queue", ctypes.c_int),
                ("fake_device", ctypes.c_int), ("fake_free_bytes", i64)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", i64), ("rejected", i64), ("completed", i64), ("queued", i64),
                ("running", i64), ("batches", i64), ("mean_batch", ctypes.c_double),
                ("algorithmic_bytes", i64), ("budget_bytes", i64), ("in_use_bytes", i64),
                ("peak_in_use_bytes", i64), ("span_s", ctypes.c_double),
                ("throughput_gbps", ctypes.c_double), ("p50_us", ctypes.c_double),
                ("p99_us", ctypes.c_double), ("max_us", ctypes.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


def request_array(count):
    """A zeroed numpy array laid out exactly as `count` ttx_request structs, with
    fields problem_dtype, n, perm, size, alpha, beta, A, B_in, B, arrival_ns,
    keep_result (outer sizes unused: contiguous tensors)."""
    import numpy as np
    P = Problem
    off = lambda f: getattr(P, f).offset
    dt = np.dtype({"names": ["dtype", "n", "perm", "size", "alpha", "beta", "A", "B_in", "B",
                             "arrival_ns", "keep_result"],
                   "formats": [np.int32, np.int32, (np.int32, MAX_DIMS), (np.int64, MAX_DIMS),
                               np.float64, np.float64, np.uint64, np.uint64, np.uint64, np.int64,
                               np.int32],
                   "offsets": [off("dtype"), off("n"), off("perm"), off("size"), off("alpha"),
                               off("beta"), off("A"), off("B_in"), off("B"),
                               Request.arrival_ns.offset, Request.keep_result.offset],
                   "itemsize": ctypes.sizeof(Request)})
    return np.zeros(count, dtype=dt)


def make_problem(dtype, perm, size, alpha, A, beta, B, outer_a=None, outer_b=None, B_in=None):
    """A ttx_problem (A, B, B_in are device addresses)."""
    q = Problem()
    q.dtype = dtype
    q.n = len(perm)
    for k, v in enumerate(perm):
        q.perm[k] = int(v)
    for k, v in enumerate(size):
        q.size[k] = int(v)
    if outer_a is not None:
        q.has_outer_a = 1
        for k, v in enumerate(outer_a):
            q.outer_a[k] = int(v)
    if outer_b is not None:
        q.has_outer_b = 1
        for k, v in enumerate(outer_b):
            q.outer_b[k] = int(v)
    alpha, beta = complex(alpha), complex(beta)
    q.alpha, q.beta = alpha.real, beta.real
    q.alpha_im, q.beta_im = alpha.imag, beta.imag
    q.A, q.B, q.B_in = A, B, B_in
    return q


_lib = None


def lib():
    """The loaded libttx.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        try:   # share the HIP runtime torch loads (one runtime per process)
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libttx.so is not built (run paper_1607_01249_amd/build.py); "
                               "there is no fallback implementation")
        L = ctypes.CDLL(LIB_PATH)
        _declare(L)
        _lib = L
    return _lib


def _declare(L):
    S = ctypes.c_int
    dp = ctypes.POINTER(ctypes.c_double)
    sig = {
        "ttx_status_string": ([S], ctypes.c_char_p),
        "ttx_last_error": ([], ctypes.c_char_p),
        "ttx_version": ([], ctypes.c_char_p),
        "ttx_transpose": ([S, S, ip, i64p, i64p, i64p, ctypes.c_double, vp, ctypes.c_double, vp, vp], S),
        "ttx_transpose_c": ([S, S, ip, i64p, i64p, i64p, dp, vp, dp, vp, vp], S),
        "ttx_plan_create": ([ctypes.POINTER(vp), S, S, ip, i64p, i64p, i64p], S),
        "ttx_plan_execute": ([vp, ctypes.c_double, vp, ctypes.c_double, vp, vp], S),
        "ttx_plan_execute_split": ([vp, ctypes.c_double, vp, ctypes.c_double, vp, vp, vp], S),
        "ttx_plan_execute_c": ([vp, dp, vp, dp, vp, vp, vp], S),
        "ttx_plan_describe": ([vp, ctypes.POINTER(PlanInfo)], S),
        "ttx_plan_set_config": ([vp, S, ctypes.POINTER(Config)], S),
        "ttx_plan_destroy": ([vp], S),
        "ttx_plan_kernel_name": ([vp, ctypes.c_double, vp, vp, ctypes.c_char_p, S], S),
        "ttx_plan_specialise": ([vp, S, S, ip], S),
        "ttx_set_auto_specialise": ([S], S),
        "ttx_transpose_cache_info": ([ip, ip], S),
        "ttx_plan_specialised_source": ([vp, S, ctypes.c_char_p, S], S),
        "ttx_tune": ([S, S, ip, i64p, i64p, i64p, S, S, S, ctypes.POINTER(Config), ip], S),
        "ttx_tune_specialised": ([S, S, ip, i64p, i64p, i64p, S, S, S, ctypes.POINTER(Config), ip], S),
        "ttx_tune_candidates": ([S, S, ip, i64p, i64p, i64p, S, ctypes.POINTER(Config),
                                 ctypes.POINTER(ctypes.c_double), S, ip], S),
        "ttx_tune_variants": ([S, S, ip, i64p, i64p, i64p, ctypes.POINTER(Config), ctypes.POINTER(Config),
                               S, ip], S),
        "ttx_tile_shapes": ([S, S, S, ip, ip, S, ip], S),
        "ttx_tune_table_save": ([ctypes.c_char_p], S),
        "ttx_tune_table_load": ([ctypes.c_char_p], S),
        "ttx_tune_table_clear": ([], S),
        "ttx_tune_table_size": ([], S),
        "ttx_tune_db_attach": ([ctypes.c_char_p], S),
        "ttx_tune_db_detach": ([], S),
        "ttx_batch_create": ([ctypes.POINTER(vp), S, ctypes.POINTER(Problem)], S),
        "ttx_batch_tune": ([vp, S, S], S),
        "ttx_batch_execute": ([vp, vp], S),
        "ttx_batch_execute_direct": ([vp, vp], S),
        "ttx_batch_update": ([vp, S, ctypes.POINTER(Problem), vp], S),
        "ttx_batch_get_info": ([vp, ctypes.POINTER(BatchInfo)], S),
        "ttx_batch_config": ([vp, S, ctypes.POINTER(Config)], S),
        "ttx_batch_destroy": ([vp], S),
        "ttx_batch_plan": ([S, ctypes.POINTER(Problem), ctypes.POINTER(Config), i64p], S),
        "ttx_batch_run_static": ([S, ctypes.POINTER(Problem), vp], S),
        "ttx_server_create": ([ctypes.POINTER(vp), ctypes.POINTER(ServerOpts)], S),
        "ttx_server_submit": ([vp, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)], S),
        "ttx_server_poll": ([vp, ctypes.c_uint64, ip], S),
        "ttx_server_wait": ([vp, ctypes.c_uint64], S),
        "ttx_server_result": ([vp, ctypes.c_uint64, ctypes.POINTER(vp), ctypes.POINTER(ctypes.c_double)], S),
        "ttx_server_release": ([vp, ctypes.c_uint64], S),
        "ttx_server_drain": ([vp], S),
        "ttx_server_cancel": ([vp, ctypes.c_uint64], S),
        "ttx_server_replay": ([vp, i64, vp, i64p, ctypes.POINTER(ctypes.c_uint64)], S),
        "ttx_server_replay_clients": ([vp, i64, vp, i64p, ctypes.c_int, ctypes.POINTER(ctypes.c_uint64)], S),
        "ttx_server_get_stats": ([vp, ctypes.POINTER(ServerStats)], S),
        "ttx_server_destroy": ([vp], S),
        "ttx_replay_sequential": ([i64, vp, i64p, vp, i64, vp, ctypes.POINTER(ctypes.c_double)], S),
        "ttx_pack": ([S, S, i64, i64, i64, i64, dp, vp, vp, vp], S),
        "ttx_gemm_panels": ([S, S, i64, i64, i64, vp, vp, vp, i64, vp], S),
        "ttx_pack_tune": ([S, S, i64, i64, i64, i64, S, S], S),
        "ttx_pack_describe": ([S, S, i64, i64, i64, i64, i64p, ip, ctypes.POINTER(Config)], S),
        "ttx_contraction_create": ([ctypes.POINTER(vp), S, S, ip, i64p, S, ip, i64p, S, ip, i64p], S),
        "ttx_contraction_describe": ([vp, ctypes.POINTER(ContractionInfo)], S),
        "ttx_contraction_execute": ([vp, ctypes.c_double, vp, vp, ctypes.c_double, vp, vp, vp], S),
        "ttx_contraction_destroy": ([vp], S),
        "ttx_copy_kernel": ([vp, vp, i64, vp], S),
        "ttx_axpby_kernel": ([S, i64, ctypes.c_double, vp, ctypes.c_double, vp, vp], S),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res


def _check(status):
    if status != OK:
        detail = lib().ttx_last_error().decode()
        raise TTXError(status, detail or lib().ttx_status_string(status).decode())
    return status


def _ints(vals, ctype=ctypes.c_int):
    if vals is None:
        return None
    vals = [int(v) for v in vals]
    return (ctype * max(1, len(vals)))(*vals)


def _i64s(vals):
    return _ints(vals, ctypes.c_int64)


# -- raw entry points -------------------------------------------------------------------
def ttx_transpose(dtype, n, perm, size, outer_a, outer_b, alpha, A, beta, B, stream=0):
    return _check(lib().ttx_transpose(dtype, n, _ints(perm), _i64s(size), _i64s(outer_a),
                                      _i64s(outer_b), float(alpha), A, float(beta), B, stream))


def _complex2(v):
    v = complex(v)
    return (ctypes.c_double * 2)(v.real, v.imag)


def ttx_transpose_c(dtype, n, perm, size, outer_a, outer_b, alpha, A, beta, B, stream=0):
    return _check(lib().ttx_transpose_c(dtype, n, _ints(perm), _i64s(size), _i64s(outer_a),
                                        _i64s(outer_b), _complex2(alpha), A, _complex2(beta), B,
                                        stream))


def ttx_plan_create(dtype, perm, size, outer_a=None, outer_b=None):
    h = vp()
    _check(lib().ttx_plan_create(ctypes.byref(h), dtype, len(perm), _ints(perm), _i64s(size),
                                 _i64s(outer_a), _i64s(outer_b)))
    return h


def ttx_plan_execute(plan, alpha, A, beta, B, stream=0):
    return _check(lib().ttx_plan_execute(plan, float(alpha), A, float(beta), B, stream))


def ttx_plan_execute_split(plan, alpha, A, beta, B_in, B_out, stream=0):
    return _check(lib().ttx_plan_execute_split(plan, float(alpha), A, float(beta), B_in, B_out, stream))


def ttx_plan_execute_c(plan, alpha, A, beta, B_in, B_out, stream=0):
    return _check(lib().ttx_plan_execute_c(plan, _complex2(alpha), A, _complex2(beta), B_in, B_out,
                                           stream))


def ttx_plan_describe(plan):
    info = PlanInfo()
    _check(lib().ttx_plan_describe(plan, ctypes.byref(info)))
    n = info.n
    return dict(dtype=info.dtype, family=FAMILY_NAMES[info.family], n=n,
                perm=list(info.perm[:n]), size=list(info.size[:n]),
                stride_a=list(info.stride_a[:n]), stride_b=list(info.stride_b[:n]),
                elements=info.elements, extent_a_bytes=info.extent_a_bytes,
                extent_b_bytes=info.extent_b_bytes,
                config=[info.config[0].as_dict(), info.config[1].as_dict()],
                config_raw=[info.config[0], info.config[1]],
                config_from_table=list(info.config_from_table),
                specialised=list(info.specialised))


def ttx_plan_set_config(plan, beta_is_zero, config):
    return _check(lib().ttx_plan_set_config(plan, int(beta_is_zero), ctypes.byref(config)))


def ttx_plan_kernel_name(plan, beta, A, B):
    buf = ctypes.create_string_buffer(256)
    _check(lib().ttx_plan_kernel_name(plan, float(beta), A, B, buf, 256))
    return buf.value.decode()


def ttx_plan_specialise(plan, beta_is_zero, reps=0):
    """Compiles and attaches the plan's size-specialised kernel; with reps > 0
    only when it times faster than the generic kernel.  Returns True when a
    kernel was attached."""
    kept = ctypes.c_int(0)
    _check(lib().ttx_plan_specialise(plan, int(bool(beta_is_zero)), int(reps), ctypes.byref(kept)))
    return bool(kept.value)


def ttx_set_auto_specialise(calls):
    return _check(lib().ttx_set_auto_specialise(int(calls)))


def ttx_transpose_cache_info():
    plans, spec = ctypes.c_int(0), ctypes.c_int(0)
    _check(lib().ttx_transpose_cache_info(ctypes.byref(plans), ctypes.byref(spec)))
    return plans.value, spec.value


def ttx_plan_specialised_source(plan, beta_is_zero):
    buf = ctypes.create_string_buffer(1 << 16)
    _check(lib().ttx_plan_specialised_source(plan, int(bool(beta_is_zero)), buf, 1 << 16))
    return buf.value.decode()


def ttx_plan_destroy(plan):
    return _check(lib().ttx_plan_destroy(plan))


def ttx_tune(dtype, perm, size, outer_a=None, outer_b=None, beta_is_zero=False,
             max_candidates=0, reps=3):
    best = Config()
    timed = ctypes.c_int(0)
    _check(lib().ttx_tune(dtype, len(perm), _ints(perm), _i64s(size), _i64s(outer_a),
                          _i64s(outer_b), int(beta_is_zero), int(max_candidates), int(reps),
                          ctypes.byref(best), ctypes.byref(timed)))
    return best, timed.value


def ttx_tune_specialised(dtype, perm, size, outer_a=None, outer_b=None, beta_is_zero=False,
                         max_candidates=0, reps=3):
    best = Config()
    timed = ctypes.c_int(0)
    _check(lib().ttx_tune_specialised(dtype, len(perm), _ints(perm), _i64s(size), _i64s(outer_a),
                                      _i64s(outer_b), int(beta_is_zero), int(max_candidates), int(reps),
                                      ctypes.byref(best), ctypes.byref(timed)))
    return best, timed.value


def ttx_tune_candidates(dtype, perm, size, outer_a=None, outer_b=None, max_candidates=0, cap=256):
    out = (Config * cap)()
    cost = (ctypes.c_double * cap)()
    count = ctypes.c_int(0)
    _check(lib().ttx_tune_candidates(dtype, len(perm), _ints(perm), _i64s(size), _i64s(outer_a),
                                     _i64s(outer_b), int(max_candidates), out, cost, cap,
                                     ctypes.byref(count)))
    return [out[i] for i in range(count.value)], [cost[i] for i in range(count.value)]


def ttx_tune_variants(dtype, perm, size, base, outer_a=None, outer_b=None, cap=64):
    """Workgroup variants (threads per workgroup x LDS row padding) of one config, itself first."""
    out = (Config * cap)()
    count = ctypes.c_int(0)
    _check(lib().ttx_tune_variants(dtype, len(perm), _ints(perm), _i64s(size), _i64s(outer_a), _i64s(outer_b),
                                   ctypes.byref(base), out, cap, ctypes.byref(count)))
    return [out[i] for i in range(count.value)]


def ttx_tune_table_save(path):
    return _check(lib().ttx_tune_table_save(path.encode()))


def ttx_tune_table_load(path):
    return _check(lib().ttx_tune_table_load(path.encode()))


def ttx_tune_table_clear():
    return _check(lib().ttx_tune_table_clear())


def ttx_tune_table_size():
    return lib().ttx_tune_table_size()


def ttx_tune_db_attach(path):
    return _check(lib().ttx_tune_db_attach(path.encode()))


def ttx_tune_db_detach():
    return _check(lib().ttx_tune_db_detach())


def _problem_array(problems):
    arr = (Problem * max(1, len(problems)))()
    for i, q in enumerate(problems):
        arr[i] = q
    return arr


def ttx_batch_create(problems):
    h = vp()
    _check(lib().ttx_batch_create(ctypes.byref(h), len(problems), _problem_array(problems)))
    return h


def ttx_batch_tune(batch, max_candidates=0, reps=3):
    return _check(lib().ttx_batch_tune(batch, int(max_candidates), int(reps)))


def ttx_batch_execute(batch, stream=0):
    return _check(lib().ttx_batch_execute(batch, stream))


def ttx_batch_execute_direct(batch, stream=0):
    return _check(lib().ttx_batch_execute_direct(batch, stream))


def ttx_batch_update(batch, problems, stream=0):
    return _check(lib().ttx_batch_update(batch, len(problems), _problem_array(problems), stream))


def ttx_batch_get_info(batch):
    info = BatchInfo()
    _check(lib().ttx_batch_get_info(batch, ctypes.byref(info)))
    return dict(count=info.count, grid=info.grid, variants_used=info.variants_used,
                tuned=info.tuned, total_tiles=info.total_tiles,
                algorithmic_bytes=info.algorithmic_bytes, chunks=info.chunks, per_call=info.per_call)


def ttx_batch_config(batch, index):
    c = Config()
    _check(lib().ttx_batch_config(batch, int(index), ctypes.byref(c)))
    return c


def ttx_batch_destroy(batch):
    return _check(lib().ttx_batch_destroy(batch))


STATIC_BATCH_MAX = 1024   # TTX_STATIC_BATCH_MAX


def ttx_batch_run_static(problems, stream=0):
    """Allocation-free batched run (the work block is a static device array)."""
    return _check(lib().ttx_batch_run_static(len(problems), _problem_array(problems), stream))


def ttx_batch_plan(problems):
    """Host-only planning of a batch: (configs, tiles) per problem."""
    n = len(problems)
    cfg = (Config * max(1, n))()
    tiles = (i64 * max(1, n))()
    _check(lib().ttx_batch_plan(n, _problem_array(problems), cfg, tiles))
    return [cfg[i] for i in range(n)], [tiles[i] for i in range(n)]


def ttx_server_create(hbm_fraction=0.8, arena_bytes=0, slots=0, max_batch=0, max_batch_bytes=0,
                      max_queue=0, fake_device=False, fake_free_bytes=0):
    o = ServerOpts(hbm_fraction, arena_bytes, slots, max_batch, max_batch_bytes, max_queue,
                   int(fake_device), fake_free_bytes)
    h = vp()
    _check(lib().ttx_server_create(ctypes.byref(h), ctypes.byref(o)))
    return h


def make_request(problem, arrival_ns=0, keep_result=False):
    return Request(problem, int(arrival_ns), int(keep_result))


def ttx_server_submit(server, request):
    t = ctypes.c_uint64(0)
    _check(lib().ttx_server_submit(server, ctypes.byref(request), ctypes.byref(t)))
    return t.value


def ttx_server_poll(server, ticket):
    d = ctypes.c_int(0)
    _check(lib().ttx_server_poll(server, ticket, ctypes.byref(d)))
    return bool(d.value)


def ttx_server_wait(server, ticket):
    return _check(lib().ttx_server_wait(server, ticket))


def ttx_server_result(server, ticket):
    b = vp()
    lat = ctypes.c_double(0)
    _check(lib().ttx_server_result(server, ticket, ctypes.byref(b), ctypes.byref(lat)))
    return b.value, lat.value


def ttx_server_release(server, ticket):
    return _check(lib().ttx_server_release(server, ticket))


def ttx_server_drain(server):
    return _check(lib().ttx_server_drain(server))


def ttx_server_cancel(server, ticket):
    """Withdraws a request that has not been launched."""
    return _check(lib().ttx_server_cancel(server, ticket))


def ttx_server_replay(server, requests, offsets_ns):
    """requests: a request_array(); offsets_ns: int64 numpy array.  Returns tickets."""
    return ttx_server_replay_clients(server, requests, offsets_ns, 1)


def ttx_server_replay_clients(server, requests, offsets_ns, clients):
    """The replay from `clients` submitting threads.  Returns tickets."""
    import numpy as np
    offsets_ns = np.ascontiguousarray(offsets_ns, dtype=np.int64)
    tickets = np.zeros(len(requests), dtype=np.uint64)
    tp = tickets.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))
    if clients == 1:
        _check(lib().ttx_server_replay(server, len(requests), requests.ctypes.data,
                                       offsets_ns.ctypes.data_as(i64p), tp))
    else:
        _check(lib().ttx_server_replay_clients(server, len(requests), requests.ctypes.data,
                                               offsets_ns.ctypes.data_as(i64p), int(clients), tp))
    return tickets


def ttx_server_get_stats(server):
    st = ServerStats()
    _check(lib().ttx_server_get_stats(server, ctypes.byref(st)))
    return st.as_dict()


def ttx_replay_sequential(requests, offsets_ns, scratch, scratch_bytes, stream=0):
    """Per-call baseline of a trace; returns the latencies in microseconds."""
    import numpy as np
    offsets_ns = np.ascontiguousarray(offsets_ns, dtype=np.int64)
    lat = np.zeros(len(requests), dtype=np.float64)
    _check(lib().ttx_replay_sequential(len(requests), requests.ctypes.data,
                                       offsets_ns.ctypes.data_as(i64p), scratch, int(scratch_bytes),
                                       stream, lat.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return lat


def ttx_server_destroy(server):
    return _check(lib().ttx_server_destroy(server))


def ttx_copy_kernel(src, dst, nbytes, stream=0):
    return _check(lib().ttx_copy_kernel(src, dst, int(nbytes), stream))


def ttx_gemm_panels(dtype, panel, m, n, k, Pa, Pb, C, ldc, stream=0):
    """C (m x n, column-major, ldc) = A * B from matrix-core operand panels."""
    return _check(lib().ttx_gemm_panels(dtype, int(panel), int(m), int(n), int(k), Pa, Pb, C, int(ldc), stream))


def ttx_tile_shapes(dtype, family, run_time_only=False):
    """[(tile_a, tile_b)] of a family's pre-compiled menu, or of its run-time-only large tiles."""
    count = ctypes.c_int()
    _check(lib().ttx_tile_shapes(dtype, family, int(bool(run_time_only)), None, None, 0, ctypes.byref(count)))
    ta = (ctypes.c_int * max(1, count.value))()
    tb = (ctypes.c_int * max(1, count.value))()
    _check(lib().ttx_tile_shapes(dtype, family, int(bool(run_time_only)), ta, tb, count.value, ctypes.byref(count)))
    return [(ta[i], tb[i]) for i in range(count.value)]


def ttx_contraction_create(dtype, labels_a, size_a, labels_b, size_b, labels_c, size_c):
    """A transpose-transpose-GEMM-transpose contraction plan (host only)."""
    h = vp()
    _check(lib().ttx_contraction_create(ctypes.byref(h), dtype, len(labels_a), _ints(labels_a), _i64s(size_a),
                                        len(labels_b), _ints(labels_b), _i64s(size_b),
                                        len(labels_c), _ints(labels_c), _i64s(size_c)))
    return h


def ttx_contraction_describe(plan):
    info = ContractionInfo()
    _check(lib().ttx_contraction_describe(plan, ctypes.byref(info)))
    return dict(m=info.m, n=info.n, k=info.k, panel=info.panel, transposed_a=bool(info.transposed_a),
                transposed_b=bool(info.transposed_b), pack_kind_a=info.pack_kind_a, pack_kind_b=info.pack_kind_b,
                order_m=list(info.order_m[:info.n_m]), order_n=list(info.order_n[:info.n_n]),
                order_k=list(info.order_k[:info.n_k]), workspace_bytes=info.workspace_bytes)


def ttx_contraction_execute(plan, alpha, A, B, beta, C, workspace, stream=0):
    return _check(lib().ttx_contraction_execute(plan, float(alpha), A, B, float(beta), C, workspace, stream))


def ttx_contraction_destroy(plan):
    return _check(lib().ttx_contraction_destroy(plan))


def ttx_pack(dtype, kind, rows, cols, ld, panel, alpha, A, P, stream=0):
    return _check(lib().ttx_pack(dtype, kind, int(rows), int(cols), int(ld), int(panel),
                                 _complex2(alpha), A, P, stream))


def ttx_pack_tune(dtype, kind, rows, cols, ld, panel, max_candidates=0, reps=3):
    return _check(lib().ttx_pack_tune(dtype, kind, int(rows), int(cols), int(ld), int(panel),
                                      int(max_candidates), int(reps)))


def ttx_pack_describe(dtype, kind, rows, cols, ld, panel):
    """(packed element count, [configs of the transpositions run])."""
    n = i64(0)
    parts = ctypes.c_int(0)
    cfg = (Config * 2)()
    _check(lib().ttx_pack_describe(dtype, kind, int(rows), int(cols), int(ld), int(panel),
                                   ctypes.byref(n), ctypes.byref(parts), cfg))
    return n.value, [cfg[i] for i in range(parts.value)]


def ttx_axpby_kernel(dtype, n, alpha, x, beta, y, stream=0):
    return _check(lib().ttx_axpby_kernel(dtype, int(n), float(alpha), x, float(beta), y, stream))


# -- torch convenience ------------------------------------------------------------------
def dtype_code(t):
    import torch
    if t.dtype == torch.float32:
        return F32
    if t.dtype == torch.float64:
        return F64
    if t.dtype == torch.complex64:
        return C32
    if t.dtype == torch.complex128:
        return C64
    raise TypeError("ttx supports float32, float64, complex64 and complex128 tensors, got %s"
                    % t.dtype)


def current_stream():
    import torch
    return torch.cuda.current_stream().cuda_stream


def transpose(A, B, perm, size, alpha=1.0, beta=0.0, outer_a=None, outer_b=None, stream=None):
    """B_{Pi(i)} <- alpha*A_i + beta*B_{Pi(i)} on device tensors used as flat
    column-major storage (Eqn. 1); asynchronous on ``stream`` (default: the
    current torch stream)."""
    pair = (dtype_code(A), dtype_code(B))
    if pair not in CODE_OF:
        raise TypeError("A and B must have the same dtype or differ only in precision")
    code = CODE_OF[pair]
    if not (A.is_cuda and B.is_cuda):
        raise ValueError("A and B must be device tensors")
    if stream is None:
        stream = current_stream()
    if isinstance(alpha, complex) or isinstance(beta, complex):
        return ttx_transpose_c(code, len(perm), perm, size, outer_a, outer_b, alpha, A.data_ptr(),
                               beta, B.data_ptr(), stream)
    return ttx_transpose(code, len(perm), perm, size, outer_a, outer_b, alpha, A.data_ptr(), beta,
                         B.data_ptr(), stream)
