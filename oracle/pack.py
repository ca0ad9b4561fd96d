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

Matrix-core operand panels (pack_mfma) are the layout a 64-lane matrix
fused multiply-add instruction of an AMD CDNA GPU reads its operands in:
for a panel of `panel` rows (left operand; columns for the right operand)
and kb = 64 / panel values of the reduction index k per instruction, lane
l of the wave holds element (l mod panel, l div panel) of the
panel x kb block of one instruction; successive instructions take
successive blocks of kb values of k.  A panel is therefore stored as its
blocks one after another, each block as 64 consecutive elements in lane
order, and the k extent is padded with zeros to a whole block:

* left operand (m x k matrix A, panels of `panel` rows):
  P[l + 64*b + p*panel*K] = alpha * A[(p*panel + l mod panel) + (b*kb + l div panel)*ld]
  with K = kb * ceil(k / kb), zero where the row is >= m or the k index >= k;
* right operand (k x n matrix A, panels of `panel` columns):
  P[l + 64*b + p*panel*K] = alpha * A[(b*kb + l div panel) + (p*panel + l mod panel)*ld]
  with the same K, zero where the column is >= n or the k index >= k.
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


LANES = 64   # lanes of a wave: one operand element each per matrix instruction


def pack_mfma(kind, A, rows, cols, ld, panel, alpha=1.0, out_dtype=None):
    """Matrix-core operand panels of the column-major rows x cols matrix in
    the flat array A (leading dimension ld): kind ROWS packs the left
    operand (rows x k, k = cols), COLS the right one (k x cols, k = rows);
    panel must divide 64.  Returns a flat array of
    ceil(extent/panel) * panel * K elements of out_dtype."""
    if LANES % panel:
        raise ValueError("panel must divide 64")
    out_dtype = np.dtype(out_dtype or A.dtype)
    kb = LANES // panel                         # k values per instruction
    split, k = (rows, cols) if kind == ROWS else (cols, rows)
    npanels = -(-split // panel)
    K = kb * -(-k // kb)                        # k padded to whole blocks
    P = np.zeros(npanels * panel * K, dtype=out_dtype)
    if split == 0 or k == 0:
        return P
    lane, blk, p = np.meshgrid(np.arange(LANES), np.arange(K // kb), np.arange(npanels), indexing="ij")
    inner = p * panel + lane % panel            # the row (ROWS) or column (COLS) of A
    kk = blk * kb + lane // panel               # the reduction index
    dst = lane + LANES * blk + p * panel * K
    src = inner + kk * ld if kind == ROWS else kk + inner * ld
    keep = (inner < split) & (kk < k)
    P[dst[keep]] = _scale(A[src[keep]], alpha, out_dtype)
    return P
