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


# -- matrix-core operand panels and the GEMM that reads them ------------------------------
def _gpu_pack_mfma(kind, A, rows, cols, ld, panel, alpha, out_dtype):
    split, k = (rows, cols) if kind == ttx.PACK_MFMA_A else (cols, rows)
    kb = 64 // panel
    n_out = -(-split // panel) * panel * (kb * -(-k // kb))
    dA, pa = to_device(A)
    dP, pp = to_device(np.full(n_out, np.nan, dtype=out_dtype))
    ttx.ttx_pack(dtype_code(A.dtype, out_dtype), kind, rows, cols, ld, panel, alpha, pa, pp, ttx.current_stream())
    out = from_device(dP)
    del dA, dP
    return out


MFMA_SHAPES = [  # rows, cols, ld, panel: ragged panels, k not a whole block, ld > rows
    (37, 13, 40, 16), (64, 32, 64, 16), (5, 3, 9, 16), (100, 7, 101, 32), (33, 66, 33, 32), (16, 1, 16, 64),
    (3, 300, 3, 8)]


@pytest.mark.parametrize("kind", [ttx.PACK_MFMA_A, ttx.PACK_MFMA_B], ids=["left", "right"])
@pytest.mark.parametrize("types", [(F32, F32), (F64, F64), (F32, F64), (C64, C64)], ids=["s", "d", "sd", "z"])
def test_mfma_panels_match_oracle(kind, types):
    """The matrix-core layout (k padded with zeros to whole blocks) element
    by element against the pinned oracle, with every padding position
    overwritten (the output starts as NaN)."""
    da, db = types
    okind = pack_oracle.ROWS if kind == ttx.PACK_MFMA_A else pack_oracle.COLS
    alpha = complex(0.75, -1.25) if db in (C32, C64) else 1.3
    for rows, cols, ld, panel in MFMA_SHAPES:
        A = workloads.uniform(ld * cols, da, seed=rows + 7 * cols)
        want = pack_oracle.pack_mfma(okind, A, rows, cols, ld, panel, alpha=alpha, out_dtype=db)
        got = _gpu_pack_mfma(kind, A, rows, cols, ld, panel, alpha, db)
        assert_parity(got, want, exact=False, what=(rows, cols, ld, panel))
        want1 = pack_oracle.pack_mfma(okind, A, rows, cols, ld, panel, out_dtype=db)
        assert_parity(_gpu_pack_mfma(kind, A, rows, cols, ld, panel, 1.0, db), want1, exact=True)


@pytest.mark.parametrize("dtype,panel", [(F32, 16), (F32, 32), (F64, 16)])
def test_gemm_reads_mfma_panels_directly(dtype, panel):
    """Packed panels go to the matrix-core GEMM as they are (no transposition
    in between): integer-valued A and B give C = A @ B exactly, with ragged
    panels, a k that is not a whole block and ldc > m; C outside m x n is
    not touched."""
    import torch
    rng = np.random.default_rng(17 + panel)
    for m, n, k, lda, ldb, ldc in [(200, 72, 96, 203, 100, 210), (37, 21, 13, 40, 15, 37), (1, 1, 1, 1, 1, 1),
                                   (64, 96, 130, 64, 131, 70)]:
        A = rng.integers(-8, 9, size=lda * k).astype(dtype)
        B = rng.integers(-8, 9, size=ldb * n).astype(dtype)
        Am = A.reshape(k, lda).T[:m].astype(np.float64)
        Bm = B.reshape(n, ldb).T[:k].astype(np.float64)
        PA = _gpu_pack_mfma(ttx.PACK_MFMA_A, A, m, k, lda, panel, 1.0, dtype)
        PB = _gpu_pack_mfma(ttx.PACK_MFMA_B, B, k, n, ldb, panel, 1.0, dtype)
        dA = torch.from_numpy(PA).cuda()
        dB = torch.from_numpy(PB).cuda()
        dC = torch.full((ldc * n,), 7.0, dtype=dA.dtype, device="cuda")
        ttx.ttx_gemm_panels(dtype_code(dtype), panel, m, n, k, dA.data_ptr(), dB.data_ptr(), dC.data_ptr(), ldc,
                            ttx.current_stream())
        torch.cuda.synchronize()
        C = dC.cpu().numpy().reshape(n, ldc).T
        assert np.array_equal(C[:m].astype(np.float64), Am @ Bm), (m, n, k)
        assert (C[m:] == 7.0).all()



@pytest.mark.parametrize("dtype,panel,mnk", [(F32, 16, (2053, 2050, 37)), (F32, 32, (4100, 4097, 9)),
                                             (F64, 16, (2053, 2049, 21)), (F32, 32, (1600, 1600, 1600)),
                                             (F64, 16, (333, 301, 701)), (F32, 16, (100, 37, 1003)),
                                             (F32, 32, (40, 70, 250))],
                         ids=["s16-2x2", "s32-2x2", "d16-2x2", "s32-deep", "d16-deep", "s16-deep", "s32-deep-small"])
def test_gemm_large_grids(dtype, panel, mnk):
    """Grids large enough for 2 x 2 blocks per wave (with ragged edges in
    both directions and a k that is not a whole chunk of blocks), and deep k
    on small grids with one block per wave (ragged panels, k not a whole
    number of chunks): integer-valued operands, C compared exactly."""
    import torch
    m, n, k = mnk
    rng = np.random.default_rng(m + n + k)
    A = rng.integers(-3, 4, size=m * k).astype(dtype)
    B = rng.integers(-3, 4, size=k * n).astype(dtype)
    PA = _gpu_pack_mfma(ttx.PACK_MFMA_A, A, m, k, m, panel, 1.0, dtype)
    PB = _gpu_pack_mfma(ttx.PACK_MFMA_B, B, k, n, k, panel, 1.0, dtype)
    dA = torch.from_numpy(PA).cuda()
    dB = torch.from_numpy(PB).cuda()
    ldc = m + 3
    dC = torch.full((ldc * n,), 7.0, dtype=dA.dtype, device="cuda")
    ttx.ttx_gemm_panels(dtype_code(dtype), panel, m, n, k, dA.data_ptr(), dB.data_ptr(), dC.data_ptr(), ldc,
                        ttx.current_stream())
    torch.cuda.synchronize()
    C = dC.cpu().numpy().reshape(n, ldc).T
    want = A.reshape(k, m).T.astype(np.float64) @ B.reshape(n, k).T.astype(np.float64)
    assert np.array_equal(C[:m].astype(np.float64), want)
    assert (C[m:] == 7.0).all()
