"""numpy mirror of the oracle (Eqn. 1), written with array views.

TEST INFRASTRUCTURE ONLY (see the package docstring).  The definition is
the same as the C oracle's, realised differently: A's outer tensor is
reshaped column-major, the addressed sub-tensor is sliced out, and
``np.transpose(sub, perm)`` produces the tensor laid out in B's index order
(gather reading: B position k holds A index ``perm[k]``, Sec. 2.1).  numpy
rounds each elementwise product and sum separately in the array's dtype.
For the complex dtypes numpy's own complex product is used, whose internal
rounding order (and use of fused multiply-add) numpy does not fix: complex
results agree with the C oracle to within a few units in the last place,
not bit for bit.
"""
import numpy as np


def _sub(flat, outer, extent):
    count = int(np.prod(outer, dtype=np.int64))
    full = flat[:count].reshape(tuple(int(o) for o in outer), order="F")
    return full[tuple(slice(0, int(e)) for e in extent)]


def transpose_np(perm, size, alpha, A, beta, B, outer_a=None, outer_b=None):
    """B <- alpha * Pi(A) + beta * B on flat host arrays, in place (Eqn. 1).

    When beta (rounded to the element type) is zero, B is not read.
    """
    perm = [int(p) for p in perm]
    size = [int(s) for s in size]
    size_b = [size[p] for p in perm]
    outer_a = list(size) if outer_a is None else [int(o) for o in outer_a]
    outer_b = list(size_b) if outer_b is None else [int(o) for o in outer_b]
    t = B.dtype.type
    a_sub = _sub(A, outer_a, size)
    b_sub = _sub(B, outer_b, size_b)
    moved = np.transpose(a_sub, perm).astype(B.dtype)   # mixed precision: to B's type first
    if np.iscomplexobj(B):
        alpha_t, beta_t = t(complex(alpha)), t(complex(beta))
    else:
        alpha_t, beta_t = t(alpha), t(beta)
    if beta_t == 0:
        b_sub[...] = alpha_t * moved
    else:
        b_sub[...] = alpha_t * moved + beta_t * b_sub
    return 0
