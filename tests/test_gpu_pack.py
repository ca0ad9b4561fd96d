"""GPU parity for GEMM operand packing (Sec. 2.1, Fig. 3) through the C ABI
against the packing oracle, and the packed panels feeding a GEMM on the
device."""
import numpy as np
import pytest

import oracle.pack as pack_oracle
import paper_1607_01249_amd as ttx
import workloads
from gpu_util import C32, C64, F32, F64, assert_parity, dtype_code, from_device, to_device

pytestmark = pytest.mark.gpu

SHAPES = [  # rows, cols, ld, panel
    (37, 19, 40, 8), (64, 33, 64, 16), (5, 3, 9, 8), (1000, 7, 1001, 6), (257, 129, 300, 12),
    (16, 1, 16, 4), (3, 300, 3, 1),
]
TYPES = [(F32, F32), (F64, F64), (C32, C32), (C64, C64), (F32, F64), (F64, F32), (C32, C64), (C64, C32)]


def _gpu_pack(kind, A, rows, cols, ld, panel, alpha, out_dtype, pad_p=0):
    split, other = (rows, cols) if kind == ttx.PACK_ROWS else (cols, rows)
    n_out = -(-split // panel) * panel * other
    dA, pa = to_device(A)
    dP, pp = to_device(np.full(n_out, np.nan, dtype=out_dtype), pad_p)
    ttx.ttx_pack(dtype_code(A.dtype, out_dtype), kind, rows, cols, ld, panel, alpha, pa, pp,
                 ttx.current_stream())
    out = from_device(dP, pad_p)
    del dA, dP
    return out


@pytest.mark.parametrize("kind", [ttx.PACK_ROWS, ttx.PACK_COLS], ids=["rows", "cols"])
@pytest.mark.parametrize("types", TYPES, ids=["s", "d", "c", "z", "sd", "ds", "cz", "zc"])
def test_pack_matches_oracle(kind, types):
    da, db = types
    alpha = complex(0.75, -1.25) if db in (C32, C64) else 1.3
    for rows, cols, ld, panel in SHAPES:
        A = workloads.uniform(ld * cols, da, seed=rows + cols)
        want = pack_oracle.pack(kind, A, rows, cols, ld, panel, alpha=alpha, out_dtype=db)
        got = _gpu_pack(kind, A, rows, cols, ld, panel, alpha, db)
        assert_parity(got, want, exact=False, what=(rows, cols, ld, panel))
        got1 = _gpu_pack(kind, A, rows, cols, ld, panel, 1.0, db)
        assert_parity(got1, pack_oracle.pack(kind, A, rows, cols, ld, panel, out_dtype=db), exact=True)


def test_pack_misaligned_output_takes_element_paths():
    A = workloads.uniform(40 * 19, F32, seed=5)
    for kind in (ttx.PACK_ROWS, ttx.PACK_COLS):
        want = pack_oracle.pack(kind, A, 37, 19, 40, 8)
        got = _gpu_pack(kind, A, 37, 19, 40, 8, 1.0, F32, pad_p=1)
        assert_parity(got, want, exact=True)


@pytest.mark.parametrize("dtype", [F32, F64])
def test_packed_panels_feed_a_gemm(dtype):
    """Rows panels of A and columns panels of B, multiplied panel by panel
    with torch on the device, give A @ B exactly (integer-valued data)."""
    import torch
    rng = np.random.default_rng(9)
    m, k, n, mr, nr, lda, ldb = 200, 96, 72, 16, 8, 203, 100
    A = rng.integers(-8, 9, size=lda * k).astype(dtype)
    B = rng.integers(-8, 9, size=ldb * n).astype(dtype)
    Am = A.reshape(k, lda).T[:m]
    Bm = B.reshape(n, ldb).T[:k]
    PA = _gpu_pack(ttx.PACK_ROWS, A, m, k, lda, mr, 1.0, dtype)
    PB = _gpu_pack(ttx.PACK_COLS, B, k, n, ldb, nr, 1.0, dtype)
    tA = torch.from_numpy(PA).cuda().view(-1, k, mr)      # [panel][c][i]
    tB = torch.from_numpy(PB).cuda().view(-1, k, nr)      # [panel][r][j]
    # block (p, q) of C = A panel p (mr x k) @ B panel q (k x nr)
    left = tA.transpose(1, 2).contiguous().reshape(-1, k)             # (panels*mr) x k
    right = tB.permute(1, 0, 2).contiguous().reshape(k, -1)           # k x (panels*nr)
    C = torch.matmul(left, right).cpu().numpy()
    assert np.array_equal(C[:m, :n], Am @ Bm)
    assert not C[m:].any() and not C[:, n:].any()


def test_pack_tune_then_pack():
    A = workloads.uniform(1000 * 64, F32, seed=11)
    ttx.ttx_pack_tune(ttx.F32, ttx.PACK_ROWS, 1000, 64, 1000, 16, max_candidates=16, reps=2)
    _, cfgs = ttx.ttx_pack_describe(ttx.F32, ttx.PACK_ROWS, 1000, 64, 1000, 16)
    assert len(cfgs) == 2
    want = pack_oracle.pack(ttx.PACK_ROWS, A, 1000, 64, 1000, 16)
    got = _gpu_pack(ttx.PACK_ROWS, A, 1000, 64, 1000, 16, 1.0, F32)
    assert_parity(got, want, exact=True)
