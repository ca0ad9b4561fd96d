"""CPU oracle for Eqn. 1 (out-of-place tensor transposition with scaling and
update, column-major, per-index leading dimensions).

TEST INFRASTRUCTURE ONLY.  Two independent CPU references live here:

* ``transpose`` -- the plain C nested loop in ``ttx_ref.c`` (loaded with
  ctypes from ``libttxref.so``, built by ``oracle/build.py``);
* ``ref_np.transpose_np`` -- the same definition written with numpy views
  (``np.transpose``'s ``axes`` argument is exactly the gather reading of the
  permutation used throughout).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It imports nothing from the library
under test, and the library imports nothing from it.
"""
import ctypes
import os

import numpy as np

from .ref_np import transpose_np  # noqa: F401  (re-exported)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libttxref.so")

OK, EINVAL, EPERM, EOVERLAP, EUNSUPPORTED = 0, 1, 2, 3, 4
DTYPES = {np.dtype(np.float32): 0, np.dtype(np.float64): 1,
          np.dtype(np.complex64): 2, np.dtype(np.complex128): 3}

_lib = None


def lib():
    """Loads (building first if absent) the C oracle."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build
            build.build()
        _lib = _load(LIB_PATH)
    return _lib


def _load(path):
    L = ctypes.CDLL(path)
    i64p = ctypes.POINTER(ctypes.c_int64)
    ip = ctypes.POINTER(ctypes.c_int)
    L.ttx_ref_transpose.argtypes = [ctypes.c_int, ctypes.c_int, ip, i64p, i64p, i64p,
                                    ctypes.c_double, ctypes.c_void_p, ctypes.c_double,
                                    ctypes.c_void_p]
    L.ttx_ref_transpose.restype = ctypes.c_int
    d2 = ctypes.POINTER(ctypes.c_double)
    L.ttx_ref_transpose_c.argtypes = [ctypes.c_int, ctypes.c_int, ip, i64p, i64p, i64p, d2,
                                      ctypes.c_void_p, d2, ctypes.c_void_p]
    L.ttx_ref_transpose_c.restype = ctypes.c_int
    L.ttx_ref_transpose_x.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ip, i64p, i64p, i64p,
                                      d2, ctypes.c_void_p, d2, ctypes.c_void_p]
    L.ttx_ref_transpose_x.restype = ctypes.c_int
    L.ttx_ref_check_x.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ip, i64p, i64p, i64p,
                                  ctypes.c_void_p, ctypes.c_void_p]
    L.ttx_ref_check_x.restype = ctypes.c_int
    L.ttx_ref_sample_c.argtypes = [ctypes.c_int, ctypes.c_int, ip, i64p, i64p, i64p, d2,
                                   ctypes.c_void_p, d2, ctypes.c_void_p, ctypes.c_int64, i64p,
                                   ctypes.c_void_p]
    L.ttx_ref_sample_c.restype = ctypes.c_int
    L.ttx_ref_check.argtypes = [ctypes.c_int, ctypes.c_int, ip, i64p, i64p, i64p,
                                ctypes.c_void_p, ctypes.c_void_p]
    L.ttx_ref_check.restype = ctypes.c_int
    L.ttx_ref_sample.argtypes = [ctypes.c_int, ctypes.c_int, ip, i64p, i64p, i64p, ctypes.c_double,
                                 ctypes.c_void_p, ctypes.c_double, ctypes.c_void_p, ctypes.c_int64,
                                 i64p, ctypes.c_void_p]
    L.ttx_ref_sample.restype = ctypes.c_int
    L.ttx_ref_b_offsets.argtypes = [ctypes.c_int, ip, i64p, i64p, ctypes.c_int64, i64p, i64p]
    L.ttx_ref_b_offsets.restype = ctypes.c_int
    L.ttx_ref_threads.argtypes = []
    L.ttx_ref_threads.restype = ctypes.c_int
    L.ttx_ref_set_threads.argtypes = [ctypes.c_int]
    L.ttx_ref_set_threads.restype = ctypes.c_int
    return L


def _arr(vals, ctype):
    if vals is None:
        return None
    vals = [int(v) for v in vals]
    return (ctype * max(1, len(vals)))(*vals)


def _scalar2(v):
    v = complex(v)
    return (ctypes.c_double * 2)(v.real, v.imag)


def transpose(perm, size, alpha, A, beta, B, outer_a=None, outer_b=None, library=None):
    """B <- alpha * Pi(A) + beta * B in place on host numpy arrays (Eqn. 1).

    ``A`` and ``B`` are flat numpy arrays (float32, float64, complex64 or
    complex128) holding the column-major outer tensors; ``perm`` is the
    gather permutation (B position k holds A index ``perm[k]``).  ``alpha``
    and ``beta`` may be complex for the complex dtypes.  A and B may differ
    in precision (float32 with float64, complex64 with complex128: mixed
    precision, computed in B's precision after converting A).  Returns the
    C status code.
    """
    L = library or lib()
    assert A.dtype in DTYPES and B.dtype in DTYPES
    assert A.flags.c_contiguous and B.flags.c_contiguous and B.flags.writeable
    n = len(perm)
    return L.ttx_ref_transpose_x(DTYPES[A.dtype], DTYPES[B.dtype], n, _arr(perm, ctypes.c_int),
                                 _arr(size, ctypes.c_int64), _arr(outer_a, ctypes.c_int64),
                                 _arr(outer_b, ctypes.c_int64), _scalar2(alpha),
                                 A.ctypes.data, _scalar2(beta), B.ctypes.data)


def check(dtype_code, perm, size, outer_a=None, outer_b=None, a_addr=1 << 20, b_addr=1 << 40,
          n=None, library=None, dtype_a=None):
    """Status code of the oracle's argument validation (touches no memory);
    ``dtype_a`` (default: ``dtype_code``) is A's type for mixed precision."""
    L = library or lib()
    n = len(perm) if n is None else n
    return L.ttx_ref_check_x(dtype_code if dtype_a is None else dtype_a, dtype_code, n,
                             _arr(perm, ctypes.c_int) if perm is not None else None,
                             _arr(size, ctypes.c_int64) if size is not None else None,
                             _arr(outer_a, ctypes.c_int64), _arr(outer_b, ctypes.c_int64),
                             a_addr, b_addr)


def sample(perm, size, alpha, A, beta, B_in, b_index, outer_a=None, outer_b=None, library=None):
    """Eqn. 1 at the B-linear sub-tensor positions ``b_index`` (int64 array);
    returns (expected values, their offsets inside B's outer tensor)."""
    L = library or lib()
    assert B_in is None or B_in.dtype == A.dtype, "sampling takes one element type"
    b_index = np.ascontiguousarray(b_index, dtype=np.int64)
    out = np.empty(len(b_index), dtype=A.dtype)
    off = np.empty(len(b_index), dtype=np.int64)
    i64p = ctypes.POINTER(ctypes.c_int64)
    st = L.ttx_ref_sample_c(DTYPES[A.dtype], len(perm), _arr(perm, ctypes.c_int),
                            _arr(size, ctypes.c_int64), _arr(outer_a, ctypes.c_int64),
                            _arr(outer_b, ctypes.c_int64), _scalar2(alpha), A.ctypes.data,
                            _scalar2(beta), B_in.ctypes.data if B_in is not None else None,
                            len(b_index), b_index.ctypes.data_as(i64p), out.ctypes.data)
    assert st == OK, st
    st = L.ttx_ref_b_offsets(len(perm), _arr(perm, ctypes.c_int), _arr(size, ctypes.c_int64),
                             _arr(outer_b, ctypes.c_int64), len(b_index),
                             b_index.ctypes.data_as(i64p), off.ctypes.data_as(i64p))
    assert st == OK, st
    return out, off


def threads(library=None):
    """OpenMP threads the oracle's loop nest runs on."""
    return (library or lib()).ttx_ref_threads()


def set_threads(n, library=None):
    """Runs later oracle calls on ``n`` OpenMP threads; returns the count now in effect."""
    return (library or lib()).ttx_ref_set_threads(int(n))
