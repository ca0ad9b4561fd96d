"""Pins the CPU oracle to facts other than itself (CPU only).

Each ``pin_*`` function takes a loaded oracle library and raises
AssertionError when the oracle disagrees with what the paper or the
mathematics fixes:

* the Sec. 2.1 example, written out by hand (tests/golden);
* a closed form: with A's values encoding their own multi-index, every B
  element must encode the A index the gather reading sends to it;
* numpy's ``transpose`` (a library routine) on every permutation of up to 5
  indices with tiny extents, contiguous and inside larger outer tensors;
* the 2D case against a textbook matrix transpose (numpy ``.T``);
* round trip through the inverse permutation, and composition of two
  permutations (which separates the gather from the scatter reading);
* the update against a separate elementwise axpby, beta = 0 never reading B,
  the non-fused operation order (contraction detector), special values;
* mixed precision (sd, ds, cz, zc): widening is exact, narrowing rounds to
  nearest on float midpoints, and any update equals numpy's conversion
  followed by the one-type transposition;
* complex elements (the c and z types): with real scalars the result equals
  the real transposition of the interleaved (re, im) planes, multiplying by
  i swaps and negates parts exactly, numpy's complex arithmetic agrees to a
  few units in the last place, and exact rational arithmetic stays within
  the rounding-error bound of the stated operation order.

``test_pins_catch_planted_mistakes`` compiles deliberately broken copies of
the oracle and checks that some pin fails for each of them.
"""
import itertools
import json
import os
import shutil
import tempfile
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import build as oracle_build
from oracle.ref_np import transpose_np

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
F32, F64 = np.dtype(np.float32), np.dtype(np.float64)
C32, C64 = np.dtype(np.complex64), np.dtype(np.complex128)
REAL_OF = {C32: F32, C64: F64}


def _golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def _elems(dims):
    return int(np.prod([int(d) for d in dims], dtype=np.int64))


def _rand(n, dtype, rng):
    dtype = np.dtype(dtype)
    if dtype in REAL_OF:
        parts = _rand(2 * n, REAL_OF[dtype], rng)
        return parts.view(dtype)
    if dtype == F32:
        return rng.random(n, dtype=np.float32) * 2 - 1
    return rng.random(n) * 2 - 1


def _run(L, perm, size, alpha, A, beta, B, outer_a=None, outer_b=None):
    st = oracle.transpose(perm, size, alpha, A, beta, B, outer_a, outer_b, library=L)
    assert st == oracle.OK, st
    return B


def _bits(x):
    if x.dtype in REAL_OF:
        x = x.view(REAL_OF[x.dtype])
    return x.view(np.uint32 if x.dtype == F32 else np.uint64)


def _same_bits(x, y):
    return np.array_equal(_bits(x), _bits(y))


def _inverse(perm):
    inv = [0] * len(perm)
    for k, p in enumerate(perm):
        inv[p] = k
    return tuple(inv)


# ---------------------------------------------------------------------------------------
def pin_sec21_example(L):
    g = _golden("sec21_merge_example.json")
    size = g["size"]
    i0, i1, i2 = np.meshgrid(*[np.arange(s) for s in size], indexing="ij")
    A = (i0 + 10 * i1 + 100 * i2).astype(np.float64).flatten(order="F")
    B = np.full(_elems(size), -1.0)
    _run(L, g["perm"], size, 1.0, A, 0.0, B)
    assert B.tolist() == [float(v) for v in g["B_flat_column_major"]]


def pin_index_encoding(L):
    """Closed form: A_i = sum_m i_m 8^m  =>  B_j = sum_k j_k 8^perm[k] (gather reading)."""
    for perm, size in [((2, 0, 3, 1), (2, 3, 4, 5)), ((1, 2, 0), (3, 4, 5)),
                       ((4, 0, 3, 1, 2), (2, 3, 2, 4, 3)), ((0, 5, 1, 4, 2, 3), (2, 2, 3, 2, 3, 2))]:
        n = len(size)
        grids = np.meshgrid(*[np.arange(s) for s in size], indexing="ij")
        A = sum(g * 8 ** m for m, g in enumerate(grids)).astype(np.float64).flatten(order="F")
        size_b = [size[p] for p in perm]
        B = np.zeros(_elems(size))
        _run(L, perm, size, 1.0, A, 0.0, B)
        jg = np.meshgrid(*[np.arange(s) for s in size_b], indexing="ij")
        expect = sum(jg[k] * 8 ** perm[k] for k in range(n)).astype(np.float64).flatten(order="F")
        assert np.array_equal(B, expect), (perm, size)


def _outer(rng, dims, pad):
    return tuple(int(d) + int(rng.integers(0, pad + 1)) for d in dims)


def pin_brute_force_vs_numpy(L, max_n=5, extents=(1, 2, 3, 5), sample_per_perm=2):
    """Every permutation of 1..max_n indices, tiny extents, contiguous and embedded."""
    rng = np.random.default_rng(11)
    for n in range(1, max_n + 1):
        for perm in itertools.permutations(range(n)):
            for _ in range(sample_per_perm):
                size = tuple(int(rng.choice(extents)) for _ in range(n))
                size_b = [size[p] for p in perm]
                for embedded in (False, True):
                    oa = _outer(rng, size, 2) if embedded else None
                    ob = _outer(rng, size_b, 2) if embedded else None
                    for dtype in (F32, F64):
                        for alpha, beta in ((1.0, 0.0), (1.3, 0.7), (-0.75, -2.0), (-1.5, 0.0)):
                            A = _rand(_elems(oa or size), dtype, rng)
                            B0 = _rand(_elems(ob or size_b), dtype, rng)
                            B1, B2 = B0.copy(), B0.copy()
                            _run(L, perm, size, alpha, A, beta, B1, oa, ob)
                            transpose_np(perm, size, alpha, A, beta, B2, oa, ob)
                            assert _same_bits(B1, B2), (perm, size, oa, ob, dtype, alpha, beta)


def pin_textbook_2d(L):
    rng = np.random.default_rng(12)
    for dtype in (F32, F64):
        m, n = 37, 53
        A = _rand(m * n, dtype, rng)
        B = _rand(n * m, dtype, rng)
        t = np.dtype(dtype).type
        Am = A.reshape((m, n), order="F")
        Bm = B.reshape((n, m), order="F")
        expect = (t(1.5) * Am.T + t(-0.25) * Bm).flatten(order="F")
        _run(L, (1, 0), (m, n), 1.5, A, -0.25, B)
        assert _same_bits(B, expect)
        # leading dimensions: the matrix is the top-left block of larger arrays
        lda, ldb = 41, 60
        A2 = _rand(lda * n, dtype, rng)
        B2 = _rand(ldb * m, dtype, rng)
        ref = B2.copy().reshape((ldb, m), order="F")
        ref[:n, :m] = A2.reshape((lda, n), order="F")[:m, :].T
        _run(L, (1, 0), (m, n), 1.0, A2, 0.0, B2, (lda, n), (ldb, m))
        assert _same_bits(B2, ref.flatten(order="F"))


def pin_round_trip(L):
    rng = np.random.default_rng(13)
    for perm, size in [((2, 0, 3, 1), (3, 4, 5, 6)), ((0, 5, 1, 4, 2, 3), (2, 3, 2, 4, 3, 2)),
                       ((1, 2, 0), (7, 1, 9)), ((4, 3, 2, 1, 0), (2, 3, 4, 3, 2))]:
        for dtype in (F32, F64):
            A = _rand(_elems(size), dtype, rng)
            T = np.zeros_like(A)
            _run(L, perm, size, 1.0, A, 0.0, T)
            size_b = [size[p] for p in perm]
            back = np.zeros_like(A)
            _run(L, _inverse(perm), size_b, 1.0, T, 0.0, back)
            assert _same_bits(back, A), (perm, size)


def pin_composition(L):
    """T_{p2}(T_{p1}(A)) == T_{r}(A) with r[k] = p1[p2[k]] (gather composition)."""
    rng = np.random.default_rng(14)
    for p1, p2, size in [((2, 0, 3, 1), (1, 3, 0, 2), (2, 3, 4, 5)),
                         ((1, 2, 0), (1, 2, 0), (3, 4, 5)),
                         ((0, 5, 1, 4, 2, 3), (3, 1, 4, 0, 5, 2), (2, 3, 2, 4, 3, 2))]:
        A = _rand(_elems(size), F64, rng)
        T1 = np.zeros_like(A)
        _run(L, p1, size, 1.0, A, 0.0, T1)
        s1 = [size[p] for p in p1]
        T2 = np.zeros_like(A)
        _run(L, p2, s1, 1.0, T1, 0.0, T2)
        r = tuple(p1[p2[k]] for k in range(len(p1)))
        direct = np.zeros_like(A)
        _run(L, r, size, 1.0, A, 0.0, direct)
        assert _same_bits(T2, direct), (p1, p2)
        # the other composition order describes a different tensor for these
        # non-commuting pairs, so this pin separates the two readings
        wrong = tuple(p2[p1[k]] for k in range(len(p1)))
        if wrong != r:
            other = np.zeros_like(A)
            _run(L, wrong, size, 1.0, A, 0.0, other)
            assert not _same_bits(T2, other)


def _axpby(alpha, x, beta, y):
    """Separate elementwise y <- alpha*x + beta*y in x's dtype, non-fused."""
    t = x.dtype.type
    out = np.empty_like(y)
    np.multiply(t(alpha), x, out=out)
    tmp = np.empty_like(y)
    np.multiply(t(beta), y, out=tmp)
    np.add(out, tmp, out=out)
    return out


def pin_update_vs_axpby(L):
    rng = np.random.default_rng(15)
    for dtype in (F32, F64):
        for perm, size in [((3, 2, 1, 0), (5, 6, 7, 8)), ((0, 2, 1, 3), (9, 5, 4, 3))]:
            A = _rand(_elems(size), dtype, rng)
            B = _rand(_elems(size), dtype, rng)
            plain = np.zeros_like(A)
            _run(L, perm, size, 1.0, A, 0.0, plain)
            for alpha, beta in ((1.3, 0.7), (-2.0, 0.5), (0.0, 1.0)):
                got = B.copy()
                _run(L, perm, size, alpha, A, beta, got)
                assert _same_bits(got, _axpby(alpha, plain, beta, B)), (dtype, perm, alpha, beta)


def pin_identity_is_axpby(L):
    rng = np.random.default_rng(16)
    for dtype in (F32, F64):
        size = (4, 5, 6)
        A = _rand(120, dtype, rng)
        B = _rand(120, dtype, rng)
        got = B.copy()
        _run(L, (0, 1, 2), size, 0.5, A, -1.5, got)
        assert _same_bits(got, _axpby(0.5, A, -1.5, B))


def pin_beta_zero_does_not_read_b(L):
    rng = np.random.default_rng(17)
    for dtype in (F32, F64):
        A = _rand(60, dtype, rng)
        B = np.full(60, np.nan, dtype=dtype)
        _run(L, (2, 0, 1), (3, 4, 5), 1.0, A, 0.0, B)
        assert not np.isnan(B).any()
        B = np.full(60, np.inf, dtype=dtype)
        _run(L, (2, 0, 1), (3, 4, 5), -2.0, A, -0.0, B)
        assert np.isfinite(B).all()


def pin_contraction_detector(L):
    g = _golden("contraction.json")
    assert g["f32"]["unfused"] == 0.0
    for dtype, p in ((F32, 12), (F64, 27)):
        t = dtype.type
        alpha = 1.0 + 2.0 ** -p
        A = np.array([alpha, alpha], dtype=dtype)
        B = np.array([1.0 + 2.0 ** -(p - 1)] * 2, dtype=dtype)
        assert A[0] == t(alpha) and float(A[0]) == alpha  # exactly representable
        _run(L, (1, 0), (1, 2), alpha, A, -1.0, B)
        assert B.tolist() == [0.0, 0.0], (dtype, B)
        # the exact value (what a fused multiply-add would round), for contrast
        exact = Fraction(alpha) * Fraction(alpha) - Fraction(1.0 + 2.0 ** -(p - 1))
        assert exact == Fraction(1, 2 ** (2 * p))


def pin_special_values(L):
    for dtype in (F32, F64):
        fi = np.finfo(dtype)
        vals = np.array([0.0, -0.0, np.inf, -np.inf, fi.max, -fi.max, fi.tiny, fi.smallest_subnormal,
                         -fi.smallest_subnormal, 1.0, -1.0, np.nan], dtype=dtype)
        A = np.concatenate([vals, vals[::-1]])
        B = np.zeros_like(A)
        _run(L, (1, 0), (len(vals), 2), 1.0, A, 0.0, B)
        expect = A.reshape((len(vals), 2), order="F").T.flatten(order="F")
        fin = ~np.isnan(expect)
        assert _same_bits(B[fin], expect[fin])
        assert np.isnan(B[~fin]).all()


def pin_embedded_canaries(L):
    """A sub-tensor written into a canary-filled outer tensor equals the
    contiguous result, and no element outside the sub-tensor changes."""
    rng = np.random.default_rng(18)
    size, perm = (6, 5, 4, 3), (1, 0, 2, 3)
    oa, ob = (8, 6, 4, 5), (7, 9, 6, 3)
    size_b = [size[p] for p in perm]
    for dtype in (F32, F64):
        A_full = _rand(_elems(oa), dtype, rng)
        A_sub = A_full.reshape(oa, order="F")[tuple(slice(0, s) for s in size)].flatten(order="F")
        ref = np.zeros(_elems(size_b), dtype=dtype)
        _run(L, perm, size, 2.0, A_sub, 0.0, ref)
        canary = dtype.type(-12345.0)
        B = np.full(_elems(ob), canary, dtype=dtype)
        _run(L, perm, size, 2.0, A_full, 0.0, B, oa, ob)
        Bv = B.reshape(ob, order="F")
        inner = Bv[tuple(slice(0, s) for s in size_b)]
        assert _same_bits(inner.flatten(order="F"), ref)
        mask = np.ones(ob, dtype=bool)
        mask[tuple(slice(0, s) for s in size_b)] = False
        assert (Bv[mask] == canary).all()


def pin_validation(L):
    big = 1 << 40
    c = lambda *a, **k: oracle.check(*a, library=L, **k)
    assert c(0, (0, 1), (2, 3)) == oracle.OK
    assert c(2, (0, 1), (2, 3)) == oracle.OK                # single complex
    assert c(4, (0, 1), (2, 3)) == oracle.EINVAL            # unknown dtype
    assert c(-1, (0, 1), (2, 3)) == oracle.EINVAL
    assert c(0, (0, 0), (2, 3)) == oracle.EPERM             # repeated index
    assert c(0, (0, 2), (2, 3)) == oracle.EPERM             # out of range
    assert c(0, (1, 0), (2, -1)) == oracle.EINVAL           # negative extent
    assert c(0, (1, 0), (2, 3), outer_a=(1, 3)) == oracle.EINVAL
    assert c(0, (1, 0), (2, 3), outer_b=(3, 1)) == oracle.EINVAL   # outer_b is in B order
    assert c(0, (1, 0), (2, 3), outer_b=(3, 2)) == oracle.OK
    assert c(0, (), (), n=0) == oracle.EINVAL
    assert c(0, tuple(range(17)), (1,) * 17) == oracle.EINVAL
    assert c(0, (1, 0), (2, 3), a_addr=big, b_addr=big + 20) == oracle.EOVERLAP
    assert c(0, (1, 0), (2, 3), a_addr=big, b_addr=big + 24) == oracle.OK
    assert c(1, (1, 0), (2, 3), a_addr=big, b_addr=big + 24) == oracle.EOVERLAP
    assert c(2, (1, 0), (2, 3), a_addr=big, b_addr=big + 48) == oracle.OK        # 8-byte elements
    assert c(3, (1, 0), (2, 3), a_addr=big, b_addr=big + 88) == oracle.EOVERLAP  # 16-byte elements
    assert c(3, (1, 0), (2, 3), a_addr=big, b_addr=big + 96) == oracle.OK
    assert c(0, (1, 0), (0, 3), a_addr=big, b_addr=big) == oracle.OK   # empty: nothing to do


# ---------------------------------------------------------------------------------------
# Complex elements.

def _complex_cases():
    return [((2, 0, 3, 1), (3, 4, 2, 5), None, None),
            ((1, 0), (7, 6), (9, 6), (8, 7)),
            ((0, 2, 1), (5, 3, 4), None, None)]


def _inner_mask(outer, extent):
    mask = np.zeros(tuple(int(o) for o in outer), dtype=bool)
    mask[tuple(slice(0, int(e)) for e in extent)] = True
    return mask.flatten(order="F")


def pin_complex_real_scalars_are_planewise(L):
    """Real alpha, beta: the complex transposition is the real one applied to
    the (re, im) planes, i.e. a real transposition with one more, kept,
    leading index of extent 2."""
    rng = np.random.default_rng(31)
    for dtype in (C32, C64):
        real = REAL_OF[dtype]
        for perm, size, oa, ob in _complex_cases():
            size_b = [size[p] for p in perm]
            A = _rand(_elems(oa or size), dtype, rng)
            B0 = _rand(_elems(ob or size_b), dtype, rng)
            perm2 = (0,) + tuple(p + 1 for p in perm)
            size2 = (2,) + tuple(size)
            oa2 = None if oa is None else (2,) + tuple(oa)
            ob2 = None if ob is None else (2,) + tuple(ob)
            for alpha, beta in ((1.0, 0.0), (-1.75, 0.0), (1.3, 0.7), (0.5, -2.25)):
                got = B0.copy()
                _run(L, perm, size, alpha, A, beta, got, oa, ob)
                want = B0.view(real).copy()
                _run(L, perm2, size2, alpha, A.view(real), beta, want, oa2, ob2)
                assert _same_bits(got.view(real), want), (dtype, perm, alpha, beta)


def pin_complex_times_i(L):
    """alpha = i rotates: (re, im) -> (-im, re) exactly; beta = i adds
    i*B, i.e. re -= B.im and im += B.re, one rounding each."""
    rng = np.random.default_rng(32)
    for dtype in (C32, C64):
        for perm, size, oa, ob in _complex_cases():
            size_b = [size[p] for p in perm]
            A = _rand(_elems(oa or size), dtype, rng)
            B0 = _rand(_elems(ob or size_b), dtype, rng)
            inner = _inner_mask(ob or size_b, size_b)
            plain = B0.copy()
            _run(L, perm, size, 1.0, A, 0.0, plain, oa, ob)
            got = B0.copy()
            _run(L, perm, size, 1j, A, 0.0, got, oa, ob)
            assert np.array_equal(got.real[inner], -plain.imag[inner])
            assert np.array_equal(got.imag[inner], plain.real[inner])
            got = B0.copy()
            _run(L, perm, size, 1.0, A, 1j, got, oa, ob)
            assert np.array_equal(got.real[inner], (plain.real - B0.imag)[inner])
            assert np.array_equal(got.imag[inner], (plain.imag + B0.real)[inner])
            assert _same_bits(got[~inner], B0[~inner])


def pin_complex_vs_numpy(L):
    """numpy's complex arithmetic (whose rounding order numpy leaves open)
    agrees to within a few units in the last place, on every permutation of
    up to 4 indices."""
    rng = np.random.default_rng(33)
    for dtype in (C32, C64):
        eps = np.finfo(REAL_OF[dtype]).eps
        for n in range(1, 5):
            for perm in itertools.permutations(range(n)):
                size = tuple(int(v) for v in rng.integers(1, 5, size=n))
                size_b = [size[p] for p in perm]
                A = _rand(_elems(size), dtype, rng)
                B0 = _rand(_elems(size_b), dtype, rng)
                alpha, beta = complex(*rng.uniform(-2, 2, 2)), complex(*rng.uniform(-2, 2, 2))
                got = B0.copy()
                _run(L, perm, size, alpha, A, beta, got)
                want = B0.copy()
                transpose_np(perm, size, alpha, A, beta, want)
                tol = 16.0 * (abs(alpha) + abs(beta)) * eps
                assert np.abs(got - want).max() <= tol, (dtype, perm)


def _exact(v):
    return Fraction(float(v))


def pin_complex_error_bound(L):
    """Each part lies within the rounding-error bound of the stated order
    (two products and their difference or sum; for the update one more sum)
    around the exact complex value alpha*a + beta*b, in rationals."""
    rng = np.random.default_rng(34)
    perm, size = (2, 0, 1), (3, 2, 4)
    size_b = [size[p] for p in perm]
    for dtype in (C32, C64):
        real = REAL_OF[dtype]
        u = Fraction(1, 2 ** (np.finfo(real).nmant + 1))
        A = _rand(_elems(size), dtype, rng)
        B0 = _rand(_elems(size_b), dtype, rng)
        a_t = A.reshape(size, order="F").transpose(perm).flatten(order="F")
        for alpha, beta in ((complex(0.75, -1.25), 0j), (complex(-0.3, 0.9), complex(1.1, 0.4)),
                            (complex(0.0, 2.0), complex(-0.5, 0.0))):
            got = B0.copy()
            _run(L, perm, size, alpha, A, beta, got)
            ar, ai = _exact(real.type(alpha.real)), _exact(real.type(alpha.imag))
            br, bi = _exact(real.type(beta.real)), _exact(real.type(beta.imag))
            upd = br != 0 or bi != 0
            k = 3 if upd else 2
            bound = k * u + 3 * u * u
            for q in range(len(got)):
                xr, xi = _exact(a_t[q].real), _exact(a_t[q].imag)
                yr, yi = (_exact(B0[q].real), _exact(B0[q].imag)) if upd else (0, 0)
                re = ar * xr - ai * xi + br * yr - bi * yi
                im = ar * xi + ai * xr + br * yi + bi * yr
                s_re = abs(ar * xr) + abs(ai * xi) + abs(br * yr) + abs(bi * yi)
                s_im = abs(ar * xi) + abs(ai * xr) + abs(br * yi) + abs(bi * yr)
                assert abs(_exact(got[q].real) - re) <= bound * s_re, (dtype, alpha, beta, q)
                assert abs(_exact(got[q].imag) - im) <= bound * s_im, (dtype, alpha, beta, q)


def pin_complex_beta_zero_does_not_read_b(L):
    rng = np.random.default_rng(35)
    for dtype in (C32, C64):
        nan = np.array([complex(np.nan, np.nan)], dtype=dtype)[0]
        A = _rand(60, dtype, rng)
        B = np.full(60, nan, dtype=dtype)
        _run(L, (2, 0, 1), (3, 4, 5), complex(0.5, -1.0), A, 0.0, B)
        assert not np.isnan(B.view(REAL_OF[dtype])).any()
        if dtype == C32:   # beta = 1e-300 i rounds to zero in single precision
            B = np.full(60, nan, dtype=dtype)
            _run(L, (2, 0, 1), (3, 4, 5), 1.0, A, 1e-300j, B)
            assert not np.isnan(B.view(F32)).any()


# ---------------------------------------------------------------------------------------
# Mixed precision (A and B of one kind, different precisions: sd, ds, cz, zc).

MIXED_PAIRS = [(F32, F64), (F64, F32), (C32, C64), (C64, C32)]


def _rand_kind(n, dtype, rng):
    return _rand(n, dtype, rng)


def pin_mixed_widening_is_exact(L):
    """A single, B double (sd, cz), alpha = 1, beta = 0: B is A transposed and
    widened, exactly (numpy's transpose and astype)."""
    rng = np.random.default_rng(41)
    for da, db in ((F32, F64), (C32, C64)):
        for perm, size in [((2, 0, 1), (5, 6, 7)), ((1, 0), (9, 4)), ((0, 2, 1, 3), (3, 4, 5, 2))]:
            A = _rand_kind(_elems(size), da, rng)
            B = np.full(_elems(size), np.nan, dtype=db)
            _run(L, perm, size, 1.0, A, 0.0, B)
            want = A.reshape(size, order="F").transpose(perm).astype(db).flatten(order="F")
            assert _same_bits(B, want), (da, db, perm)


def pin_mixed_narrowing_rounds_to_nearest(L):
    """A double, B single (ds, zc), alpha = 1, beta = 0: each part rounds to
    the nearest float, ties to even (values on and beside float midpoints)."""
    u = 2.0 ** -24   # half an ulp of 1.0f
    src = [1.0 + u, 1.0 + 3 * u, 1.0 + u * (1 + 2.0 ** -20), -(1.0 + 3 * u), 2.0 ** -150,
           3.0 * 2.0 ** -150, 1e300, -1e300, 0.1]
    want = [1.0, 1.0 + 4 * u, 1.0 + 2 * u, -(1.0 + 4 * u), 0.0, 2.0 ** -148, np.inf, -np.inf,
            float.fromhex("0x1.99999ap-4")]
    A = np.array(src, dtype=F64)
    B = np.zeros(len(src), dtype=F32)
    _run(L, (0, 1), (len(src), 1), 1.0, A, 0.0, B)
    assert B.tolist() == [float(np.float32(w)) for w in want], B
    assert np.signbit(B[4]) == False   # noqa: E712
    # complex: finite values only (alpha = 1 multiplies as (1, 0), and 0 * inf is NaN)
    fin = [k for k in range(len(src)) if abs(src[k]) < 1e300]
    re, im = [src[k] for k in fin], [src[k] for k in fin[::-1]]
    Az = np.array([complex(a, b) for a, b in zip(re, im)], dtype=C64)
    Bz = np.zeros(len(fin), dtype=C32)
    _run(L, (0, 1), (len(fin), 1), 1.0, Az, 0.0, Bz)
    assert Bz.real.tolist() == B[fin].tolist() and Bz.imag.tolist() == B[fin[::-1]].tolist()


def pin_mixed_is_conversion_then_update(L):
    """Any alpha, beta: the mixed result equals A converted to B's type (numpy
    astype, round to nearest) followed by the one-type transposition."""
    rng = np.random.default_rng(42)
    for da, db in MIXED_PAIRS:
        for perm, size, oa, ob in [((2, 0, 3, 1), (3, 4, 2, 5), None, None),
                                   ((1, 0), (7, 6), (9, 6), (8, 7))]:
            size_b = [size[p] for p in perm]
            A = _rand_kind(_elems(oa or size), da, rng) * 3.7
            B0 = _rand_kind(_elems(ob or size_b), db, rng)
            cx = db in (C32, C64)
            for alpha, beta in ((1.3, 0.7), (-2.0, 0.0)) + (((0.5 - 1j), (0.25 + 2j)),) * cx:
                got = B0.copy()
                _run(L, perm, size, alpha, A, beta, got, oa, ob)
                want = B0.copy()
                _run(L, perm, size, alpha, A.astype(db), beta, want, oa, ob)
                assert _same_bits(got, want), (da, db, perm, alpha, beta)


def pin_mixed_validation(L):
    big = 1 << 40
    c = lambda *a, **k: oracle.check(*a, library=L, **k)
    for da, db in ((0, 1), (1, 0), (2, 3), (3, 2)):
        assert c(db, (1, 0), (2, 3), dtype_a=da) == oracle.OK
    for da, db in ((0, 2), (2, 0), (1, 3), (3, 1), (0, 3), (4, 0)):
        assert c(db, (1, 0), (2, 3), dtype_a=da) == oracle.EINVAL, (da, db)
    # overlap with A in 4-byte and B in 8-byte elements (6 elements each)
    assert c(1, (1, 0), (2, 3), a_addr=big, b_addr=big + 20, dtype_a=0) == oracle.EOVERLAP
    assert c(1, (1, 0), (2, 3), a_addr=big, b_addr=big + 24, dtype_a=0) == oracle.OK
    # A in 8-byte elements after B in 4-byte ones: [40, 88) meets [20, 44); [44, 92) does not
    assert c(0, (1, 0), (2, 3), a_addr=big + 40, b_addr=big + 20, dtype_a=1) == oracle.EOVERLAP
    assert c(0, (1, 0), (2, 3), a_addr=big + 44, b_addr=big + 20, dtype_a=1) == oracle.OK


PINS = [pin_sec21_example, pin_index_encoding, pin_brute_force_vs_numpy, pin_textbook_2d,
        pin_round_trip, pin_composition, pin_update_vs_axpby, pin_identity_is_axpby,
        pin_beta_zero_does_not_read_b, pin_contraction_detector, pin_special_values,
        pin_embedded_canaries, pin_validation, pin_complex_real_scalars_are_planewise,
        pin_complex_times_i, pin_complex_vs_numpy, pin_complex_error_bound,
        pin_complex_beta_zero_does_not_read_b, pin_mixed_widening_is_exact,
        pin_mixed_narrowing_rounds_to_nearest, pin_mixed_is_conversion_then_update,
        pin_mixed_validation]


@pytest.mark.parametrize("pin", PINS, ids=[p.__name__ for p in PINS])
def test_oracle_pin(pin):
    pin(oracle.lib())


def test_numpy_mirror_matches_sec21_example():
    g = _golden("sec21_merge_example.json")
    size = g["size"]
    i0, i1, i2 = np.meshgrid(*[np.arange(s) for s in size], indexing="ij")
    A = (i0 + 10 * i1 + 100 * i2).astype(np.float64).flatten(order="F")
    B = np.zeros(_elems(size))
    transpose_np(g["perm"], size, 1.0, A, 0.0, B)
    assert B.tolist() == [float(v) for v in g["B_flat_column_major"]]


# ---------------------------------------------------------------------------------------
# Planted mistakes: each line below is one plausible error in the oracle's source.
MUTANTS = {
    "scatter_reading": [("size_b[k] = size[perm[k]];", "size_b[perm[k]] = size[k];"),
                        ("a_stride_in_b_order[k] = stride_a[perm[k]];",
                         "a_stride_in_b_order[perm[k]] = stride_a[k];")],
    "dropped_beta_term": [("B[off_b] = scaled_a + scaled_b;", "B[off_b] = scaled_a;")],
    "wrong_sign": [("B[off_b] = scaled_a + scaled_b;", "B[off_b] = scaled_a - scaled_b;")],
    "fused_update": [("float scaled_b = beta * B[off_b];\n        B[off_b] = scaled_a + scaled_b;",
                      "B[off_b] = __builtin_fmaf(alpha, A[off_a], beta * B[off_b]);"),
                     ("double scaled_b = beta * B[off_b];\n        B[off_b] = scaled_a + scaled_b;",
                      "B[off_b] = __builtin_fma(alpha, A[off_a], beta * B[off_b]);")],
    "ldb_from_lda": [("int64_t o = outer_b ? outer_b[k] : size_b[k];",
                      "int64_t o = outer_a ? outer_a[k] : size_b[k];")],
    "reads_b_when_beta_zero": [("B[off_b] = alpha * A[off_a];\n",
                                "B[off_b] = alpha * A[off_a] + beta * B[off_b];\n")],
    "unpermuted_read": [("off_a += j[k] * a_stride_in_b_order[k];", "off_a += j[k] * stride_a[k];")],
    "alpha_dropped": [("B[off_b] = alpha * A[off_a];\n", "B[off_b] = A[off_a];\n")],
    "lda_reversed": [("int64_t o = outer_a ? outer_a[m] : size[m];",
                      "int64_t o = outer_a ? outer_a[n - 1 - m] : size[m];")],
    "complex_cross_sign": [("pr = t1 - t2, pi = t3 + t4;", "pr = t1 + t2, pi = t3 + t4;")],
    "complex_imag_sign": [("pr = t1 - t2, pi = t3 + t4;", "pr = t1 - t2, pi = t3 - t4;")],
    "complex_parts_swapped": [("const float xr = A[2 * off_a], xi = A[2 * off_a + 1];",
                               "const float xi = A[2 * off_a], xr = A[2 * off_a + 1];"),
                              ("const double xr = A[2 * off_a], xi = A[2 * off_a + 1];",
                               "const double xi = A[2 * off_a], xr = A[2 * off_a + 1];")],
    "complex_beta_imag_dropped": [("qr = u1 - u2, qi = u3 + u4;", "qr = u1, qi = u3;")],
    "complex_beta_real_only_test": [("if (br == 0.0f && bi == 0.0f) {", "if (br == 0.0f) {"),
                                    ("if (br == 0.0 && bi == 0.0) {", "if (br == 0.0) {")],
    "complex_unscaled_offsets": [("A[2 * off_a]", "A[off_a]"), ("A[2 * off_a + 1]", "A[off_a + 1]")],
    "mixed_not_converted": [("            if (dtype_a != dtype) {", "            if (0) {")],
    "mixed_imag_dropped": [("const double a[2] = {(double)x[0], (double)x[1]};",
                            "const double a[2] = {(double)x[0], 0.0};")],
    "mixed_offset_not_doubled": [("const float *x = (const float *)A + 2 * off_a;",
                                  "const float *x = (const float *)A + off_a;")],
    "mixed_pair_unchecked": [("    if (!ref_pair_valid(dtype_a, dtype_b))\n        return REF_EINVAL;\n", "")],
    "complex_alpha_imag_in_f32": [("const float alpha_fi = (float)alpha[1], beta_fi = (float)beta[1];",
                                   "const float alpha_fi = 0.0f, beta_fi = (float)beta[1];")],
}


def _build_mutant(tmp, name, edits):
    with open(oracle_build.SRC) as f:
        src = f.read()
    for old, new in edits:
        assert old in src, (name, old)
        src = src.replace(old, new)
    if name == "transposed_strides":   # stride over the other tensor's outer sizes
        src = src.replace("int64_t o = outer_a ? outer_a[m] : size[m];",
                          "int64_t o = outer_a ? outer_a[n - 1 - m] : size[n - 1 - m];"
                          " if (o < size[m]) o = size[m];")
    path = os.path.join(tmp, name + ".c")
    with open(path, "w") as f:
        f.write(src)
    return oracle_build.build(out=os.path.join(tmp, "lib" + name + ".so"), src=path, extra=("-w",))


def _caught_by(lib_path):
    """Names of the pins that fail against the library at lib_path."""
    L = oracle._load(lib_path)
    caught = []
    for pin in PINS:
        try:
            pin(L)
        except AssertionError:
            caught.append(pin.__name__)
    return caught


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_pins_catch_planted_mistakes():
    """Each mutant runs in a child process: some mistakes (a B stride taken
    from A's outer sizes) write outside B, which must not corrupt the test
    process.  A child that dies instead of reporting also counts as caught."""
    import subprocess
    import sys
    tmp = tempfile.mkdtemp(prefix="ttx_mutants_")
    here = os.path.dirname(os.path.abspath(__file__))
    root = os.path.dirname(here)
    try:
        for name, edits in MUTANTS.items():
            path = _build_mutant(tmp, name, edits)
            code = ("import json, sys; sys.path[:0] = [%r, %r]; import test_oracle_pins as t; "
                    "print(json.dumps(t._caught_by(%r)))" % (here, root, path))
            r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True,
                               timeout=300)
            caught = json.loads(r.stdout.strip().splitlines()[-1]) if r.returncode == 0 else ["crash"]
            assert caught, "no pin catches the planted mistake %r" % name
    finally:
        shutil.rmtree(tmp, ignore_errors=True)


def test_sampled_oracle_matches_full_oracle():
    """The one-element-at-a-time entry point agrees with the full nested loop."""
    rng = np.random.default_rng(19)
    for perm, size, oa, ob in [((2, 0, 3, 1), (5, 6, 7, 3), None, None),
                               ((1, 0, 2, 3), (6, 5, 4, 3), (8, 5, 4, 3), (7, 9, 5, 3)),
                               ((0, 2, 1), (4, 3, 5), None, (6, 5, 3))]:
        size_b = [size[p] for p in perm]
        for dtype, (alpha, beta) in itertools.product((F32, F64, C32, C64),
                                                      ((1.3, 0.7), (1.0, 0.0))):
            A = _rand(_elems(oa or size), dtype, rng)
            B0 = _rand(_elems(ob or size_b), dtype, rng)
            full = B0.copy()
            _run(oracle.lib(), perm, size, alpha, A, beta, full, oa, ob)
            idx = rng.integers(0, _elems(size), size=50)
            vals, off = oracle.sample(perm, size, alpha, A, beta, B0, idx, oa, ob)
            assert _same_bits(vals, full[off])
        for dtype, (alpha, beta) in itertools.product((C32, C64), ((0.3 - 1.2j, 0.7 + 0.25j),
                                                                   (1j, 0.0))):
            A = _rand(_elems(oa or size), dtype, rng)
            B0 = _rand(_elems(ob or size_b), dtype, rng)
            full = B0.copy()
            _run(oracle.lib(), perm, size, alpha, A, beta, full, oa, ob)
            idx = rng.integers(0, _elems(size), size=50)
            vals, off = oracle.sample(perm, size, alpha, A, beta, B0, idx, oa, ob)
            assert _same_bits(vals, full[off])


# ---------------------------------------------------------------------------------------
# GEMM operand packing (Sec. 2.1, Fig. 3): oracle/pack.py.
from oracle import pack as pack_oracle   # noqa: E402


def test_pack_oracle_tiny_example_by_hand():
    """A = [[1, 4], [2, 5], [3, 6]] (column-major 1..6), panels of 2 rows:
    panel 0 holds rows 0-1 as a 2x2 column-major block, panel 1 row 2 and a
    zero row; panels of 1 column are the columns themselves."""
    A = np.arange(1, 7, dtype=np.float64)
    P = pack_oracle.pack(pack_oracle.ROWS, A, 3, 2, 3, 2)
    assert P.tolist() == [1, 2, 4, 5, 3, 0, 6, 0]
    Q = pack_oracle.pack(pack_oracle.COLS, A, 3, 2, 3, 1)
    assert Q.tolist() == [1, 2, 3, 4, 5, 6]
    R = pack_oracle.pack(pack_oracle.COLS, A, 3, 2, 3, 2)   # one panel: rows of 2 contiguous
    assert R.tolist() == [1, 4, 2, 5, 3, 6]


def _int_matrix(rng, n, dtype):
    return rng.integers(-8, 9, size=n).astype(dtype)


def test_pack_oracle_gemm_identity():
    """Panels feed a GEMM: for rows packing of A (m x k) every panel times X
    gives its rows of A @ X; for columns packing of Y (k x n), W times every
    panel gives its columns of W @ Y (integer-valued, so the products are
    exact)."""
    rng = np.random.default_rng(71)
    for m, k, n, mr, lda in [(37, 19, 5, 8, 40), (16, 7, 3, 4, 16), (5, 3, 2, 8, 9)]:
        A = _int_matrix(rng, lda * k, np.float64)
        Am = A.reshape(k, lda).T[:m]           # column-major view with ld
        X = _int_matrix(rng, k * n, np.float64).reshape(k, n)
        P = pack_oracle.pack(pack_oracle.ROWS, A, m, k, lda, mr)
        npan = -(-m // mr)
        panels = P.reshape(npan, k, mr)        # [p][c][i]
        C = Am @ X
        for p in range(npan):
            rows = slice(p * mr, min(m, (p + 1) * mr))
            got = panels[p].T @ X              # mr x n, padded rows give zeros
            nrow = rows.stop - rows.start
            assert np.array_equal(got[:nrow], C[rows])
            assert not got[nrow:].any()
    for k, n, w, nr, ldy in [(19, 37, 5, 8, 21), (7, 16, 3, 4, 7)]:
        Y = _int_matrix(rng, ldy * n, np.float64)
        Ym = Y.reshape(n, ldy).T[:k]
        W = _int_matrix(rng, w * k, np.float64).reshape(w, k)
        P = pack_oracle.pack(pack_oracle.COLS, Y, k, n, ldy, nr)
        npan = -(-n // nr)
        panels = P.reshape(npan, k, nr)        # [p][r][j]
        C = W @ Ym
        for p in range(npan):
            cols = slice(p * nr, min(n, (p + 1) * nr))
            got = W @ panels[p]
            ncol = cols.stop - cols.start
            assert np.array_equal(got[:, :ncol], C[:, cols])
            assert not got[:, ncol:].any()


def test_pack_oracle_is_the_fig3_transposition():
    """With whole panels and ld a multiple of the panel, rows packing is the
    transposition of the view (mr, m/mr, k) with perm (0, 2, 1), and columns
    packing that of (k, nr, n/nr) with perm (1, 0, 2) (the pinned oracle)."""
    rng = np.random.default_rng(72)
    for dtype in (F32, F64, C32, C64):
        m, k, mr, lda = 24, 7, 8, 32
        A = _rand(lda * k, dtype, rng)
        P = pack_oracle.pack(pack_oracle.ROWS, A, m, k, lda, mr, alpha=0.5)
        T = np.zeros(m * k, dtype=dtype)
        _run(oracle.lib(), (0, 2, 1), (mr, m // mr, k), 0.5, A, 0.0, T, (mr, lda // mr, k))
        assert _same_bits(P, T)
        kk, n, nr, ldy = 9, 12, 4, 10
        Y = _rand(ldy * n, dtype, rng)
        P = pack_oracle.pack(pack_oracle.COLS, Y, kk, n, ldy, nr, alpha=-1.5)
        T = np.zeros(kk * n, dtype=dtype)
        _run(oracle.lib(), (1, 0, 2), (kk, nr, n // nr), -1.5, Y, 0.0, T, (ldy, nr, n // nr))
        assert _same_bits(P, T)


def test_pack_oracle_complex_and_mixed_scalars_match_the_transposition_oracle():
    rng = np.random.default_rng(73)
    for da, db in ((C32, C64), (C64, C32), (F32, F64), (F64, F32), (C64, C64)):
        m, k, mr = 16, 5, 4
        A = _rand(m * k, da, rng)
        alpha = complex(0.75, -1.25) if db in (C32, C64) else 1.3
        P = pack_oracle.pack(pack_oracle.ROWS, A, m, k, m, mr, alpha=alpha, out_dtype=db)
        T = np.zeros(m * k, dtype=db)
        _run(oracle.lib(), (0, 2, 1), (mr, m // mr, k), alpha, A, 0.0, T)
        assert _same_bits(P, T), (da, db)


# -- matrix-core operand panels (oracle/pack.py pack_mfma) ----------------------------------
def test_pack_mfma_tiny_example_by_hand():
    """A 2 x 5 left operand in one 16-row panel: four k values per block, so
    K = 8; block 0 holds columns 0..3 at lanes i + 16*c, block 1 column 4 at
    lanes 64 + i, everything else is zero."""
    A = np.array([1, 2, 3, 4, 5, 6, 7, 8, 9, 10], dtype=np.float32)   # 2 x 5, ld = 2
    P = pack_oracle.pack_mfma(pack_oracle.ROWS, A, 2, 5, 2, 16)
    want = np.zeros(16 * 8, dtype=np.float32)
    for (i, c), pos in {(0, 0): 0, (1, 0): 1, (0, 1): 16, (1, 1): 17, (0, 2): 32, (1, 2): 33,
                        (0, 3): 48, (1, 3): 49, (0, 4): 64, (1, 4): 65}.items():
        want[pos] = A[i + 2 * c]
    assert np.array_equal(P, want)
    # the same matrix as a right operand (k = 2 rows, n = 5 columns) in 32-column
    # panels: two k values per block, lane j + 32*r holds row r of column j
    Q = pack_oracle.pack_mfma(pack_oracle.COLS, A, 2, 5, 2, 32)
    want = np.zeros(32 * 2, dtype=np.float32)
    for j in range(5):
        for r in range(2):
            want[j + 32 * r] = A[r + 2 * j]
    assert np.array_equal(Q, want)


def _pad_columns(A, rows, cols, ld, cols_to):
    """The column-major matrix with zero columns appended up to cols_to (ld kept)."""
    M = np.zeros(ld * cols_to, dtype=A.dtype)
    M[:ld * (cols - 1) + rows] = A[:ld * (cols - 1) + rows]
    return M


def _pad_rows(A, rows, cols, ld, rows_to):
    """The column-major matrix with zero rows appended up to rows_to (new ld = rows_to)."""
    M = np.zeros(rows_to * cols, dtype=A.dtype)
    for c in range(cols):
        M[c * rows_to:c * rows_to + rows] = A[c * ld:c * ld + rows]
    return M


@pytest.mark.parametrize("panel", [16, 32, 64, 8])
def test_pack_mfma_is_rows_and_columns_packing_of_the_k_padded_matrix(panel):
    """The matrix-core layout is the Fig. 3 packing (pinned above) of the
    matrix with k padded by zeros to whole blocks of 64/panel values."""
    rng = np.random.default_rng(41)
    kb = 64 // panel
    for m, k, ld in [(37, 13, 40), (16, 8, 16), (5, 1, 7), (64, 30, 64), (1, 3, 1)]:
        K = kb * -(-k // kb)
        A = rng.standard_normal(ld * k).astype(np.float64)
        P = pack_oracle.pack_mfma(pack_oracle.ROWS, A, m, k, ld, panel, alpha=1.5)
        want = pack_oracle.pack(pack_oracle.ROWS, _pad_columns(A, m, k, ld, K), m, K, ld, panel, alpha=1.5)
        assert np.array_equal(P, want), (m, k, ld)
        # right operand: k rows, n columns
        n, ldb = m, max(ld, k)
        Y = rng.standard_normal(ldb * n).astype(np.float32)
        Q = pack_oracle.pack_mfma(pack_oracle.COLS, Y, k, n, ldb, panel, alpha=-0.5)
        want = pack_oracle.pack(pack_oracle.COLS, _pad_rows(Y, k, n, ldb, K), K, n, K, panel, alpha=-0.5)
        assert np.array_equal(Q, want), (k, n, ldb)


def _mfma_emulated(Pa, Pb, m, n, K, panel):
    """C = A @ B from left and right operand panels, consumed as a 64-lane
    matrix instruction reads them (the documented operand order of the
    M x N x kb FP32/FP64 instructions with M = N = panel, kb = 64/panel:
    lane l supplies A[l mod M][l div M] and B[l div N][l mod N] of the
    instruction's block).  Written from that description, not from the
    packing formula."""
    kb = 64 // panel
    mp, nq = -(-m // panel), -(-n // panel)
    C = np.zeros((mp * panel, nq * panel), dtype=np.float64)
    for p in range(mp):
        for q in range(nq):
            acc = np.zeros((panel, panel))
            for b in range(K // kb):
                a_regs = Pa[p * panel * K + 64 * b:p * panel * K + 64 * b + 64]
                b_regs = Pb[q * panel * K + 64 * b:q * panel * K + 64 * b + 64]
                Ablk = np.zeros((panel, kb))
                Bblk = np.zeros((kb, panel))
                for lane in range(64):
                    Ablk[lane % panel, lane // panel] = a_regs[lane]
                    Bblk[lane // panel, lane % panel] = b_regs[lane]
                acc += Ablk @ Bblk
            C[p * panel:(p + 1) * panel, q * panel:(q + 1) * panel] = acc
    return C[:m, :n]


@pytest.mark.parametrize("panel", [16, 32])
def test_pack_mfma_feeds_the_matrix_instruction(panel):
    """Integer matrices: the panels read in the instruction's lane order give
    A @ B exactly, with ragged panels and a k that is not a whole block."""
    rng = np.random.default_rng(43)
    for m, n, k, lda, ldb in [(37, 21, 13, 40, 15), (16, 16, 4, 16, 4), (50, 3, 7, 50, 9)]:
        A = rng.integers(-8, 9, size=lda * k).astype(np.float64)
        B = rng.integers(-8, 9, size=ldb * n).astype(np.float64)
        kb = 64 // panel
        K = kb * -(-k // kb)
        Pa = pack_oracle.pack_mfma(pack_oracle.ROWS, A, m, k, lda, panel)
        Pb = pack_oracle.pack_mfma(pack_oracle.COLS, B, k, n, ldb, panel)
        Am = A.reshape(k, lda).T[:m, :k]
        Bm = B.reshape(n, ldb).T[:k, :n]
        assert np.array_equal(_mfma_emulated(Pa, Pb, m, n, K, panel), Am @ Bm), (m, n, k)
        # a transposed operand order (lane l holding element (l div kb, l mod kb))
        # would not: check that the emulator tells the two apart
        if m >= panel and k >= kb and (m, k) != (kb, panel):
            bad = Pa.copy()
            blk = bad[:64].reshape(panel, kb).T.reshape(-1)   # swap the roles of lane bits
            bad[:64] = blk
            assert not np.array_equal(_mfma_emulated(bad, Pb, m, n, K, panel), Am @ Bm)


def test_pack_mfma_empty_and_argument_errors():
    A = np.zeros(4, dtype=np.float32)
    assert pack_oracle.pack_mfma(pack_oracle.ROWS, A, 0, 4, 1, 16).size == 0
    assert pack_oracle.pack_mfma(pack_oracle.COLS, A, 0, 3, 1, 16).size == 0
    with pytest.raises(ValueError):
        pack_oracle.pack_mfma(pack_oracle.ROWS, A, 2, 2, 2, 12)
