"""Helpers for the GPU parity tests: run the HIP library through its C ABI on
device copies of host arrays, and compare results with the oracle's."""
import numpy as np

import paper_1607_01249_amd as ttx

F32, F64 = np.dtype(np.float32), np.dtype(np.float64)
C32, C64 = np.dtype(np.complex64), np.dtype(np.complex128)
REAL_OF = {C32: F32, C64: F64}
_CODES = {F32: ttx.F32, F64: ttx.F64, C32: ttx.C32, C64: ttx.C64}
_DTYPES = {v: k for k, v in _CODES.items()}
# data-type code -> (A's numpy dtype, B's numpy dtype)
TYPES_OF_CODE = {code: (_DTYPES[a], _DTYPES[b]) for (a, b), code in ttx.CODE_OF.items()}


def dtype_code(dtype, dtype_b=None):
    """The ttx data-type code for A's dtype (and B's, when it differs)."""
    a = _CODES[np.dtype(dtype)]
    b = a if dtype_b is None else _CODES[np.dtype(dtype_b)]
    return ttx.CODE_OF[(a, b)]


def _torch_dtype(dtype):
    import torch
    return {F32: torch.float32, F64: torch.float64, C32: torch.complex64,
            C64: torch.complex128}[np.dtype(dtype)]


def to_device(x, pad_elems=0):
    """Device copy of a host array; with pad_elems > 0 the data starts that
    many elements into the allocation (for misaligned-pointer cases).
    Returns (tensor, address of the first element)."""
    import torch
    t = torch.empty(len(x) + pad_elems, dtype=_torch_dtype(x.dtype), device="cuda")
    t[pad_elems:].copy_(torch.from_numpy(x))
    return t, t.data_ptr() + pad_elems * x.dtype.itemsize


def from_device(t, pad_elems=0):
    import torch
    torch.cuda.synchronize()
    return t[pad_elems:].cpu().numpy()


def gpu_transpose(perm, size, alpha, A, beta, B, outer_a=None, outer_b=None, pad_a=0, pad_b=0,
                  plan_config=None, specialise=False):
    """Runs Eqn. 1 on the GPU through ttx_transpose (or a plan with a forced
    config, or a plan with its size-specialised kernel) and returns B as a
    host array."""
    dA, pa = to_device(A, pad_a)
    dB, pb = to_device(B, pad_b)
    stream = ttx.current_stream()
    cx = isinstance(alpha, complex) or isinstance(beta, complex)
    if plan_config is None and not specialise:
        run = ttx.ttx_transpose_c if cx else ttx.ttx_transpose
        run(dtype_code(A.dtype, B.dtype), len(perm), perm, size, outer_a, outer_b, alpha, pa, beta, pb,
            stream)
    else:
        plan = ttx.ttx_plan_create(dtype_code(A.dtype, B.dtype), perm, size, outer_a, outer_b)
        try:
            beta0 = B.dtype.type(beta) == 0
            if plan_config is not None:
                ttx.ttx_plan_set_config(plan, beta0, plan_config)
            if specialise:
                ttx.ttx_plan_specialise(plan, beta0)
                info = ttx.ttx_plan_describe(plan)
                assert info["specialised"][int(beta0)] == int(info["family"] in ("moved", "preserved"))
            if cx:
                ttx.ttx_plan_execute_c(plan, alpha, pa, beta, pb, pb, stream)
            else:
                ttx.ttx_plan_execute(plan, alpha, pa, beta, pb, stream)
        finally:
            ttx.ttx_plan_destroy(plan)
    out = from_device(dB, pad_b)
    del dA, dB
    return out


def ordered_bits(x):
    """Maps floats to integers whose order and differences count ulps."""
    if x.dtype == F32:
        i = x.view(np.int32).astype(np.int64)
        return np.where(i < 0, np.int64(-2 ** 31) - i, i)
    i = x.view(np.int64)
    return np.where(i < 0, np.int64(-2 ** 63) - i, i)


def max_ulp(got, ref):
    nan_g, nan_r = np.isnan(got), np.isnan(ref)
    assert np.array_equal(nan_g, nan_r), "NaN positions differ"
    g = ordered_bits(got[~nan_g])
    r = ordered_bits(ref[~nan_r])
    diff = np.nonzero(g != r)[0]
    if diff.size == 0:
        return 0
    # exact integer arithmetic on the (few) differing elements
    return max(abs(int(g[k]) - int(r[k])) for k in diff)


def assert_parity(got, ref, exact, what=""):
    """exact: every element bit-identical (NaNs compared by class);
    otherwise at most 1 ulp apart (the same unfused operation order makes
    bit-identity the expectation; the count of differing elements is
    reported)."""
    assert got.shape == ref.shape and got.dtype == ref.dtype
    if got.dtype in REAL_OF:   # complex: both parts, compared as real numbers
        got, ref = got.view(REAL_OF[got.dtype]), ref.view(REAL_OF[ref.dtype])
    nan_g, nan_r = np.isnan(got), np.isnan(ref)
    assert np.array_equal(nan_g, nan_r), "NaN positions differ %s" % what
    ib = np.uint32 if got.dtype == F32 else np.uint64
    differ = int(np.count_nonzero(got[~nan_g].view(ib) != ref[~nan_r].view(ib)))
    if exact:
        assert differ == 0, "%d elements differ %s" % (differ, what)
    else:
        ulp = max_ulp(got, ref)
        assert ulp <= 1, "max %s ulp (%d elements differ) %s" % (ulp, differ, what)
    return differ


_hip = None


def dev_copy(dst, src, nbytes):
    """Device-to-device copy through the HIP runtime (hipMemcpy), synchronous."""
    global _hip
    import ctypes
    import torch
    if _hip is None:
        maps = open("/proc/self/maps").read().splitlines()
        paths = sorted({l.split()[-1] for l in maps if "libamdhip64" in l})
        _hip = ctypes.CDLL(paths[0])
        _hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
        _hip.hipMemcpy.restype = ctypes.c_int
    torch.cuda.synchronize()
    rc = _hip.hipMemcpy(dst, src, nbytes, 3)
    assert rc == 0, rc
