"""CPU oracle for a binary tensor contraction, the operation that Sec. 1
casts as matrix products via transpositions and that Sec. 4 names as what
the transposition is a building block for.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Definition.  A, B and C are column-major tensors (first mode fastest) with
the extents given per mode; every mode carries an integer label.  A label
that A and B carry and C does not is contracted; every label of C is
carried by exactly one of A and B (no batch labels, no label twice in one
tensor, no label in one operand only):

    C[c] <- alpha * (sum over the contracted labels of A[a] * B[b]) + beta * C[c]

where a, b and c take the values that the labels fix.  The sum is taken
exactly to float64 rounding (float64 products and sums); alpha times the
sum and beta times C are two products added in float64, rounded once to
C's type.  With beta == 0, C is not read (NaN in C stays out).

`contract` evaluates the sum with numpy's einsum on float64 copies: einsum
with explicit subscripts computes exactly this sum of products, one output
element at a time.  `magnitude` returns the same sum over |A| and |B|, the
scale of the rounding error a floating-point evaluation of the sum can make
(Higham, Accuracy and Stability of Numerical Algorithms, Sec. 3.1: a sum of
k products computed in unit roundoff u is within gamma_k * sum |a||b| of
the exact one, gamma_k = k u / (1 - k u)).
"""
import numpy as np


def check_labels(labels_a, size_a, labels_b, size_b, labels_c, size_c):
    """The extent of every label and the contracted labels (in A's order);
    raises ValueError where the definition above does not apply."""
    ext = {}
    for name, labels, size in (("A", labels_a, size_a), ("B", labels_b, size_b), ("C", labels_c, size_c)):
        if len(labels) != len(size):
            raise ValueError("%s: %d labels for %d extents" % (name, len(labels), len(size)))
        if len(set(labels)) != len(labels):
            raise ValueError("%s carries a label twice" % name)
        for l, s in zip(labels, size):
            if int(s) < 0:
                raise ValueError("negative extent")
            if ext.setdefault(l, int(s)) != int(s):
                raise ValueError("label %r has two extents" % (l,))
    sa, sb, sc = set(labels_a), set(labels_b), set(labels_c)
    for l in ext:
        n = (l in sa) + (l in sb) + (l in sc)
        if n != 2:
            raise ValueError("label %r is carried by %d tensors (must be 2)" % (l, n))
        if l in sc and l in sa and l in sb:
            raise ValueError("batch label %r" % (l,))
    return ext, [l for l in labels_a if l in sb]


def _view(T, size):
    return np.asarray(T).reshape(tuple(int(s) for s in size), order="F") if len(size) else np.asarray(T).reshape(())


def _sum_of_products(labels_a, A, size_a, labels_b, B, size_b, labels_c, size_c):
    check_labels(labels_a, size_a, labels_b, size_b, labels_c, size_c)
    ids = {l: i for i, l in enumerate(sorted(set(labels_a) | set(labels_b) | set(labels_c), key=repr))}
    a = _view(A, size_a).astype(np.float64)
    b = _view(B, size_b).astype(np.float64)
    s = np.einsum(a, [ids[l] for l in labels_a], b, [ids[l] for l in labels_b], [ids[l] for l in labels_c],
                  optimize=False)
    return np.asarray(s, dtype=np.float64).reshape(tuple(int(x) for x in size_c))


def contract(labels_a, A, size_a, labels_b, B, size_b, labels_c, size_c, alpha=1.0, beta=0.0, C=None,
             out_dtype=None):
    """C <- alpha * sum A*B + beta * C (definition above), returned as a flat
    column-major array of C's dtype (out_dtype, else A's); C (flat,
    column-major) is read only when beta != 0."""
    out_dtype = np.dtype(out_dtype if out_dtype is not None else np.asarray(A).dtype)
    s = _sum_of_products(labels_a, A, size_a, labels_b, B, size_b, labels_c, size_c)
    r = np.float64(alpha) * s
    if beta != 0:
        if C is None:
            raise ValueError("beta != 0 needs C")
        r = r + np.float64(beta) * _view(C, size_c).astype(np.float64)
    return r.reshape(-1, order="F").astype(out_dtype)


def magnitude(labels_a, A, size_a, labels_b, B, size_b, labels_c, size_c):
    """sum |A| * |B| over the contracted labels, per C element (flat, column-major, float64)."""
    s = _sum_of_products(labels_a, np.abs(np.asarray(A, dtype=np.float64)), size_a,
                         labels_b, np.abs(np.asarray(B, dtype=np.float64)), size_b, labels_c, size_c)
    return s.reshape(-1, order="F")


def contract_at(labels_a, A, size_a, labels_b, B, size_b, labels_c, size_c, positions, alpha=1.0, beta=0.0,
                C=None, out_dtype=None):
    """The same result at the given flat (column-major) positions of C only,
    one element at a time: the free labels are fixed by the position, and
    the sum runs over the contracted labels of the two slices this leaves of
    A and B.  For checking tensors too large to contract whole on the CPU."""
    ext, _ = check_labels(labels_a, size_a, labels_b, size_b, labels_c, size_c)
    out_dtype = np.dtype(out_dtype if out_dtype is not None else np.asarray(A).dtype)
    a, b = _view(A, size_a), _view(B, size_b)
    c = _view(C, size_c) if beta != 0 else None
    con = [l for l in labels_a if l in labels_b]
    ids = {l: i for i, l in enumerate(con)}
    out = np.empty(len(positions), dtype=np.float64)
    for j, pos in enumerate(positions):
        idx = np.unravel_index(int(pos), tuple(int(s) for s in size_c), order="F") if len(size_c) else ()
        val = dict(zip(labels_c, (int(i) for i in idx)))
        sa = tuple(val[l] if l in val else slice(None) for l in labels_a)
        sb = tuple(val[l] if l in val else slice(None) for l in labels_b)
        s = np.einsum(a[sa].astype(np.float64), [ids[l] for l in labels_a if l in ids],
                      b[sb].astype(np.float64), [ids[l] for l in labels_b if l in ids], [], optimize=False)
        r = np.float64(alpha) * np.float64(s)
        if beta != 0:
            r = r + np.float64(beta) * np.float64(c[idx])
        out[j] = r
    return out.astype(out_dtype)
