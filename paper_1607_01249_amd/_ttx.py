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

F32, F64 = 0, 1
OK, EINVAL, EPERM, EOVERLAP, EUNSUPPORTED, ENOMEM, EHIP, EBUSY, ENOTFOUND = range(9)
FAMILY_EMPTY, FAMILY_FLAT, FAMILY_PRESERVED, FAMILY_MOVED = range(4)
FAMILY_NAMES = {0: "empty", 1: "flat", 2: "preserved", 3: "moved"}
CFG_XCD_SWIZZLE, CFG_NT_STORE = 1, 2

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
                ("order", ctypes.c_int * MAX_DIMS), ("flags", ctypes.c_int)]

    def as_dict(self):
        return dict(family=FAMILY_NAMES[self.family], tile_a=self.tile_a, tile_b=self.tile_b,
                    threads=self.threads, order=list(self.order[:self.n_order]), flags=self.flags)


class PlanInfo(ctypes.Structure):
    _fields_ = [("dtype", ctypes.c_int), ("family", ctypes.c_int), ("n", ctypes.c_int),
                ("perm", ctypes.c_int * MAX_DIMS), ("size", i64 * MAX_DIMS),
                ("stride_a", i64 * MAX_DIMS), ("stride_b", i64 * MAX_DIMS),
                ("elements", i64), ("extent_a_bytes", i64), ("extent_b_bytes", i64),
                ("config", Config * 2), ("config_from_table", ctypes.c_int * 2)]


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
    sig = {
        "ttx_status_string": ([S], ctypes.c_char_p),
        "ttx_last_error": ([], ctypes.c_char_p),
        "ttx_version": ([], ctypes.c_char_p),
        "ttx_transpose": ([S, S, ip, i64p, i64p, i64p, ctypes.c_double, vp, ctypes.c_double, vp, vp], S),
        "ttx_plan_create": ([ctypes.POINTER(vp), S, S, ip, i64p, i64p, i64p], S),
        "ttx_plan_execute": ([vp, ctypes.c_double, vp, ctypes.c_double, vp, vp], S),
        "ttx_plan_execute_split": ([vp, ctypes.c_double, vp, ctypes.c_double, vp, vp, vp], S),
        "ttx_plan_describe": ([vp, ctypes.POINTER(PlanInfo)], S),
        "ttx_plan_set_config": ([vp, S, ctypes.POINTER(Config)], S),
        "ttx_plan_destroy": ([vp], S),
        "ttx_plan_kernel_name": ([vp, ctypes.c_double, vp, vp, ctypes.c_char_p, S], S),
        "ttx_tune": ([S, S, ip, i64p, i64p, i64p, S, S, S, ctypes.POINTER(Config), ip], S),
        "ttx_tune_candidates": ([S, S, ip, i64p, i64p, i64p, S, ctypes.POINTER(Config),
                                 ctypes.POINTER(ctypes.c_double), S, ip], S),
        "ttx_tune_table_save": ([ctypes.c_char_p], S),
        "ttx_tune_table_load": ([ctypes.c_char_p], S),
        "ttx_tune_table_clear": ([], S),
        "ttx_tune_table_size": ([], S),
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


def ttx_plan_create(dtype, perm, size, outer_a=None, outer_b=None):
    h = vp()
    _check(lib().ttx_plan_create(ctypes.byref(h), dtype, len(perm), _ints(perm), _i64s(size),
                                 _i64s(outer_a), _i64s(outer_b)))
    return h


def ttx_plan_execute(plan, alpha, A, beta, B, stream=0):
    return _check(lib().ttx_plan_execute(plan, float(alpha), A, float(beta), B, stream))


def ttx_plan_execute_split(plan, alpha, A, beta, B_in, B_out, stream=0):
    return _check(lib().ttx_plan_execute_split(plan, float(alpha), A, float(beta), B_in, B_out, stream))


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
                config_from_table=list(info.config_from_table))


def ttx_plan_set_config(plan, beta_is_zero, config):
    return _check(lib().ttx_plan_set_config(plan, int(beta_is_zero), ctypes.byref(config)))


def ttx_plan_kernel_name(plan, beta, A, B):
    buf = ctypes.create_string_buffer(256)
    _check(lib().ttx_plan_kernel_name(plan, float(beta), A, B, buf, 256))
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


def ttx_tune_candidates(dtype, perm, size, outer_a=None, outer_b=None, max_candidates=0, cap=256):
    out = (Config * cap)()
    cost = (ctypes.c_double * cap)()
    count = ctypes.c_int(0)
    _check(lib().ttx_tune_candidates(dtype, len(perm), _ints(perm), _i64s(size), _i64s(outer_a),
                                     _i64s(outer_b), int(max_candidates), out, cost, cap,
                                     ctypes.byref(count)))
    return [out[i] for i in range(count.value)], [cost[i] for i in range(count.value)]


def ttx_tune_table_save(path):
    return _check(lib().ttx_tune_table_save(path.encode()))


def ttx_tune_table_load(path):
    return _check(lib().ttx_tune_table_load(path.encode()))


def ttx_tune_table_clear():
    return _check(lib().ttx_tune_table_clear())


def ttx_tune_table_size():
    return lib().ttx_tune_table_size()


def ttx_copy_kernel(src, dst, nbytes, stream=0):
    return _check(lib().ttx_copy_kernel(src, dst, int(nbytes), stream))


def ttx_axpby_kernel(dtype, n, alpha, x, beta, y, stream=0):
    return _check(lib().ttx_axpby_kernel(dtype, int(n), float(alpha), x, float(beta), y, stream))


# -- torch convenience ------------------------------------------------------------------
def dtype_code(t):
    import torch
    if t.dtype == torch.float32:
        return F32
    if t.dtype == torch.float64:
        return F64
    raise TypeError("ttx supports float32 and float64 tensors, got %s" % t.dtype)


def current_stream():
    import torch
    return torch.cuda.current_stream().cuda_stream


def transpose(A, B, perm, size, alpha=1.0, beta=0.0, outer_a=None, outer_b=None, stream=None):
    """B_{Pi(i)} <- alpha*A_i + beta*B_{Pi(i)} on device tensors used as flat
    column-major storage (Eqn. 1); asynchronous on ``stream`` (default: the
    current torch stream)."""
    code = dtype_code(A)
    if dtype_code(B) != code:
        raise TypeError("A and B must have the same dtype")
    if not (A.is_cuda and B.is_cuda):
        raise ValueError("A and B must be device tensors")
    if stream is None:
        stream = current_stream()
    return ttx_transpose(code, len(perm), perm, size, outer_a, outer_b, alpha, A.data_ptr(), beta,
                         B.data_ptr(), stream)
