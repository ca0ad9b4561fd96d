"""CPU oracle for GEMM operand packing (Sec. 2.1, Fig. 3).

TEST INFRASTRUCTURE ONLY (see the package docstring).  Packing is the
transposition of a column-major matrix viewed as a 3D tensor whose split
index becomes (position in panel, panel number), with the panel number
moved outermost; a ragged last panel is padded with zeros.  Written here
from that definition with explicit index arithmetic:

* rows packing (left operand, panels of mr rows):
  P[i + c*mr + p*mr*cols] = alpha * A[(p*mr + i) + c*ld], zero where
  p*mr + i >= rows;
* columns packing (right operand, panels of nr columns):
  P[j + r*nr + p*nr*rows] = alpha * A[r + (p*nr + j)*ld], zero where
  p*nr + j >= cols.

Each A element is first converted to P's dtype (mixed precision: widening
exact, narrowing to nearest) and multiplied by alpha rounded to P's type,
one rounding per product; complex products follow the textbook order,
re = ar*xr - ai*xi and im = ar*xi + ai*xr, each product and sum rounded on
its own (Eqn. 1 with beta = 0, as in ttx_ref.c).
"""
import numpy as np

ROWS, COLS = 0, 1


def _scale(x, alpha, dtype):
    """alpha * x in dtype, products and sums rounded separately."""
    x = x.astype(dtype)
    if np.iscomplexobj(x):
        real = np.float32 if dtype == np.complex64 else np.float64
        a = complex(alpha)
        ar, ai = real(a.real), real(a.imag)
        xr, xi = x.real.copy(), x.imag.copy()
        t1, t2, t3, t4 = ar * xr, ai * xi, ar * xi, ai * xr
        out = np.empty(x.shape, dtype=dtype)
        out.real = t1 - t2
        out.imag = t3 + t4
        return out
    return dtype.type(alpha) * x


def pack(kind, A, rows, cols, ld, panel, alpha=1.0, out_dtype=None):
    """Packed panels of the column-major rows x cols matrix held in the flat
    array A (leading dimension ld), as a flat array of out_dtype (default:
    A's dtype)."""
    out_dtype = np.dtype(out_dtype or A.dtype)
    split, other = (rows, cols) if kind == ROWS else (cols, rows)
    npanels = -(-split // panel)
    P = np.zeros(npanels * panel * other, dtype=out_dtype)
    if split == 0 or other == 0:
        return P
    if kind == ROWS:
        i, c, p = np.meshgrid(np.arange(panel), np.arange(cols), np.arange(npanels), indexing="ij")
        row = p * panel + i
        dst = i + c * panel + p * panel * cols
        src = row + c * ld
        keep = row < rows
    else:
        j, r, p = np.meshgrid(np.arange(panel), np.arange(rows), np.arange(npanels), indexing="ij")
        col = p * panel + j
        dst = j + r * panel + p * panel * rows
        src = r + col * ld
        keep = col < cols
    P[dst[keep]] = _scale(A[src[keep]], alpha, out_dtype)
    return P
