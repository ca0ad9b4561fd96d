"""Pins of the tensor-contraction oracle (oracle/tensor_contract.py) against
what the definition and textbook special cases fix, independent of the
oracle's own einsum evaluation: pure-Python loops over every index on tiny
tensors, the matrix product, outer and inner products, all-ones closed
forms, a contraction with an identity matrix that is a transposition (the
pinned transposition oracle), the column-major reading of a hand-worked
example, and the label rules."""
import itertools

import numpy as np
import pytest

import oracle
from oracle import tensor_contract as tc

F32, F64 = np.float32, np.float64


def _brute(labels_a, A, size_a, labels_b, B, size_b, labels_c, size_c, alpha, beta, C):
    """Every C element as an explicit loop over the contracted labels (column-major offsets by hand)."""
    ext = {}
    for ls, ss in ((labels_a, size_a), (labels_b, size_b), (labels_c, size_c)):
        for l, s in zip(ls, ss):
            ext[l] = s
    con = [l for l in labels_a if l in labels_b]

    def off(labels, size, val):
        o, st = 0, 1
        for l, s in zip(labels, size):
            o += val[l] * st
            st *= s
        return o

    out = np.zeros(int(np.prod(size_c, dtype=np.int64)), dtype=np.float64)
    for cv in itertools.product(*[range(ext[l]) for l in labels_c]):
        val = dict(zip(labels_c, cv))
        s = 0.0
        for kv in itertools.product(*[range(ext[l]) for l in con]):
            val.update(zip(con, kv))
            s += float(A[off(labels_a, size_a, val)]) * float(B[off(labels_b, size_b, val)])
        o = off(labels_c, size_c, val)
        out[o] = alpha * s + (beta * float(C[o]) if beta != 0 else 0.0)
    return out


TINY = [  # labels_a, size_a, labels_b, size_b, labels_c, size_c
    ((0, 1), (3, 4), (1, 2), (4, 5), (0, 2), (3, 5)),                      # matrix product
    ((0, 5, 1, 6), (2, 3, 3, 2), (4, 6, 2, 5), (2, 2, 3, 3), (0, 1, 2, 4), (2, 3, 3, 2)),
    ((7, 3, 9), (2, 3, 4), (9, 8, 7), (4, 3, 2), (8, 3), (3, 3)),
    ((0, 1, 2), (2, 3, 2), (3,), (4,), (2, 3, 1, 0), (2, 4, 3, 2)),         # outer product
    ((0, 1), (3, 4), (1, 0), (4, 3), (), ()),                               # full contraction
    ((0, 1, 2), (2, 0, 3), (1, 3), (0, 2), (2, 0, 3), (3, 2, 2)),           # an empty contracted extent
]


@pytest.mark.parametrize("case", range(len(TINY)))
@pytest.mark.parametrize("scal", [(1.0, 0.0), (-0.75, 1.5)], ids=["a1b0", "ab"])
def test_oracle_matches_index_loops(case, scal):
    la, sa, lb, sb, lc, sc = TINY[case]
    alpha, beta = scal
    rng = np.random.default_rng(case)
    A = rng.standard_normal(int(np.prod(sa, dtype=np.int64)))
    B = rng.standard_normal(int(np.prod(sb, dtype=np.int64)))
    C = rng.standard_normal(int(np.prod(sc, dtype=np.int64)))
    got = tc.contract(la, A, sa, lb, B, sb, lc, sc, alpha, beta, C)
    want = _brute(la, A, sa, lb, B, sb, lc, sc, alpha, beta, C)
    np.testing.assert_allclose(got, want, rtol=1e-13, atol=1e-13)


def test_matrix_product_and_column_major_reading():
    """labels (i,k)(k,j)->(i,j) is A @ B for column-major flat storage; a
    hand-worked 2x2 case fixes the storage order."""
    rng = np.random.default_rng(1)
    m, k, n = 7, 5, 6
    A = rng.standard_normal(m * k)
    B = rng.standard_normal(k * n)
    got = tc.contract((0, 2), A, (m, k), (2, 1), B, (k, n), (0, 1), (m, n)).reshape(n, m).T
    want = A.reshape(k, m).T @ B.reshape(n, k).T
    np.testing.assert_allclose(got, want, rtol=1e-13)
    # A = [[1, 3], [2, 4]] (flat 1,2,3,4), B = [[5, 7], [6, 8]]: A @ B = [[23, 31], [34, 46]]
    got = tc.contract((0, 2), np.array([1., 2., 3., 4.]), (2, 2), (2, 1), np.array([5., 6., 7., 8.]), (2, 2),
                      (0, 1), (2, 2))
    assert list(got) == [23., 34., 31., 46.]
    # the same with C's labels swapped: C^T, i.e. B^T A^T
    got = tc.contract((0, 2), np.array([1., 2., 3., 4.]), (2, 2), (2, 1), np.array([5., 6., 7., 8.]), (2, 2),
                      (1, 0), (2, 2))
    assert list(got) == [23., 31., 34., 46.]


def test_outer_inner_and_all_ones():
    rng = np.random.default_rng(2)
    x, y = rng.standard_normal(6), rng.standard_normal(5)
    np.testing.assert_allclose(tc.contract((0,), x, (6,), (1,), y, (5,), (0, 1), (6, 5)),
                               np.outer(x, y).reshape(-1, order="F"), rtol=1e-15)
    np.testing.assert_allclose(tc.contract((0,), x, (6,), (0,), x, (6,), (), ()), [np.dot(x, x)], rtol=1e-13)
    # all ones: every element is alpha * (product of the contracted extents) + beta * C
    sa, sb, sc = (3, 4, 5, 2), (5, 6, 3), (4, 2, 6)
    C = np.full(48, 2.0)
    got = tc.contract((0, 1, 2, 3), np.ones(120), sa, (2, 4, 0), np.ones(90), sb, (1, 3, 4), sc, 0.5, -1.0, C)
    assert np.all(got == 0.5 * 15 - 2.0)


def test_identity_contraction_is_the_transposition():
    """C_{j,i,l} = sum_k A_{i,k,l} I_{k,j} relabels A's index k as j: the
    transposition with gather perm (1, 0, 2), scaled and updated (Eqn. 1),
    as the pinned transposition oracle computes it."""
    rng = np.random.default_rng(3)
    size = (5, 4, 3)
    A = rng.standard_normal(60)
    I = np.eye(4).reshape(-1, order="F")
    C = rng.standard_normal(60)
    got = tc.contract((0, 1, 2), A, size, (1, 9), I, (4, 4), (9, 0, 2), (4, 5, 3), 1.25, -0.5, C)
    want = C.copy()
    assert oracle.transpose((1, 0, 2), size, 1.25, A, -0.5, want) == 0
    np.testing.assert_allclose(got, want, rtol=1e-15, atol=1e-15)


def test_beta_zero_does_not_read_c_and_rounds_once():
    A = np.array([1.0, 2.0], dtype=F32)
    B = np.array([3.0, 4.0], dtype=F32)
    got = tc.contract((0,), A, (2,), (0,), B, (2,), (), (), 1.0, 0.0, np.array([np.nan], dtype=F32))
    assert got.dtype == F32 and got[0] == 11.0
    # float64 sum, one rounding to float32: 1 + 2^-30 + (-1) is 2^-30, not 0
    A = np.array([1.0, 2.0 ** -30, -1.0])
    B = np.ones(3)
    assert tc.contract((0,), A, (3,), (0,), B, (3,), (), (), out_dtype=F32)[0] == np.float32(2.0 ** -30)


def test_magnitude_bounds_a_rounded_sum():
    """A float32 sum of products stays within gamma_k * sum |a||b| of the exact one."""
    rng = np.random.default_rng(4)
    m, k, n = 9, 300, 7
    A = rng.standard_normal(m * k).astype(F32)
    B = rng.standard_normal(k * n).astype(F32)
    exact = tc.contract((0, 2), A, (m, k), (2, 1), B, (k, n), (0, 1), (m, n), out_dtype=F64)
    approx = (A.reshape(k, m).T @ B.reshape(n, k).T).astype(F32).reshape(-1, order="F")
    u = 2.0 ** -24
    bound = k * u / (1 - k * u) * tc.magnitude((0, 2), A, (m, k), (2, 1), B, (k, n), (0, 1), (m, n))
    assert np.all(np.abs(approx - exact) <= bound)
    assert np.all(bound > 0)


@pytest.mark.parametrize("bad", [
    ((0, 0), (2, 2), (0, 1), (2, 3), (1,), (3,)),          # label twice in A
    ((0, 1), (2, 2), (1, 2), (3, 3), (0, 2), (2, 3)),      # label 1 with two extents
    ((0, 1, 3), (2, 2, 2), (1, 2, 3), (2, 3, 2), (0, 2, 3), (2, 3, 2)),   # batch label
    ((0, 1, 4), (2, 2, 2), (1, 2), (2, 3), (0, 2), (2, 3)),  # label in A only
    ((0, 1), (2, 2), (1, 2), (2, 3), (0,), (2,)),          # label 2 in B only
])
def test_label_rules(bad):
    la, sa, lb, sb, lc, sc = bad
    A = np.ones(int(np.prod(sa)))
    B = np.ones(int(np.prod(sb)))
    with pytest.raises(ValueError):
        tc.contract(la, A, sa, lb, B, sb, lc, sc)


def test_planted_mistakes_are_caught():
    """A dropped alpha, a swapped C label order or a transposed operand each
    change the result of the matrix-product pin above."""
    rng = np.random.default_rng(5)
    m, k, n = 4, 3, 5
    A = rng.standard_normal(m * k)
    B = rng.standard_normal(k * n)
    ref = tc.contract((0, 2), A, (m, k), (2, 1), B, (k, n), (0, 1), (m, n), 2.0)
    assert not np.allclose(ref, tc.contract((0, 2), A, (m, k), (2, 1), B, (k, n), (0, 1), (m, n), 1.0))
    assert not np.allclose(ref, tc.contract((0, 2), A, (m, k), (2, 1), B, (k, n), (1, 0), (n, m), 2.0))
    At = A.reshape(k, m).T.reshape(-1)   # A stored row-major, read as column-major
    assert not np.allclose(ref, tc.contract((0, 2), At, (m, k), (2, 1), B, (k, n), (0, 1), (m, n), 2.0))


@pytest.mark.parametrize("case", [1, 2, 4, 5])
def test_sampled_elements_match_index_loops(case):
    """contract_at (one element at a time) against the index loops, at every position."""
    la, sa, lb, sb, lc, sc = TINY[case]
    rng = np.random.default_rng(10 + case)
    A = rng.standard_normal(int(np.prod(sa, dtype=np.int64)))
    B = rng.standard_normal(int(np.prod(sb, dtype=np.int64)))
    C = rng.standard_normal(int(np.prod(sc, dtype=np.int64)))
    n = C.size
    got = tc.contract_at(la, A, sa, lb, B, sb, lc, sc, np.arange(n), 0.5, 2.0, C)
    np.testing.assert_allclose(got, _brute(la, A, sa, lb, B, sb, lc, sc, 0.5, 2.0, C), rtol=1e-13, atol=1e-13)
