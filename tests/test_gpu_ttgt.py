"""GPU parity for the transpose-transpose-GEMM-transpose contraction
(Sec. 1, Sec. 4) through the C ABI, against the contraction oracle.

Integer-valued operands make every product and partial sum exact in both
precisions (|sum| < 2^24), so those results must equal the oracle bit for
bit.  Uniform operands are held to the error bound of a k-term sum of
products in the element type plus the roundings of the last step: at
most (k + 4) * u * (|alpha| * sum |a||b| + |beta| * |C|) per element, with
u = 2^-24 (FP32) or 2^-53 (FP64), sum |a||b| from the oracle."""
import sys

import numpy as np
import pytest

import paper_1607_01249_amd as ttx
import workloads
from gpu_util import F32, F64, dtype_code, from_device, to_device
from oracle import tensor_contract as tc

pytestmark = pytest.mark.gpu

UNIT = {F32: 2.0 ** -24, F64: 2.0 ** -53}


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _run(case, dtype, A, B, C, alpha, beta, pad_ws=0):
    """C after the contraction on the device (host arrays in, host array out)."""
    import torch
    sa, sb, sc = workloads.contraction_sizes(case)
    plan = ttx.ttx_contraction_create(dtype_code(dtype), case["labels_a"], sa, case["labels_b"], sb,
                                      case["labels_c"], sc)
    try:
        info = ttx.ttx_contraction_describe(plan)
        dA, pa = to_device(A) if A.size else (None, 0)
        dB, pb = to_device(B) if B.size else (None, 0)
        dC, pc = to_device(C) if C.size else (None, 0)
        ws = torch.full((info["workspace_bytes"] // 4 + 64 + pad_ws,), float("nan"), dtype=torch.float32,
                        device="cuda")
        ttx.ttx_contraction_execute(plan, alpha, pa, pb, beta, pc, ws.data_ptr() + 4 * pad_ws,
                                    ttx.current_stream())
        out = from_device(dC) if C.size else C.copy()
        del dA, dB, dC, ws
        return out, info
    finally:
        ttx.ttx_contraction_destroy(plan)


def _inputs(case, dtype, seed, integer):
    sizes = workloads.contraction_sizes(case)
    n = [int(np.prod(s, dtype=np.int64)) for s in sizes]
    if integer:
        rng = np.random.default_rng(seed)
        return [rng.integers(-4, 5, size=x).astype(dtype) for x in n]
    return [workloads.uniform(x, dtype, seed + i) for i, x in enumerate(n)]


def _bound(case, dtype, A, B, C, alpha, beta):
    sa, sb, sc = workloads.contraction_sizes(case)
    mag = tc.magnitude(case["labels_a"], A, sa, case["labels_b"], B, sb, case["labels_c"], sc)
    k = int(np.prod([case["extent"][l] for l in case["labels_a"] if l in case["labels_b"]], dtype=np.int64))
    return (k + 4) * UNIT[dtype] * (abs(alpha) * mag + abs(beta) * np.abs(C.astype(np.float64)))


SCALARS = [(1.0, 0.0), (-0.75, 1.5)]


@pytest.mark.parametrize("case", workloads.CONTRACTION_PARITY, ids=lambda c: c["name"])
@pytest.mark.parametrize("dtype", [F32, F64], ids=["f32", "f64"])
def test_contraction_matches_oracle(case, dtype):
    sa, sb, sc = workloads.contraction_sizes(case)
    la, lb, lc = case["labels_a"], case["labels_b"], case["labels_c"]
    for alpha, beta in SCALARS:
        # exact: integer-valued operands
        A, B, C = _inputs(case, dtype, 3, integer=True)
        got, info = _run(case, dtype, A, B, C, alpha, beta)
        want = tc.contract(la, A, sa, lb, B, sb, lc, sc, alpha, beta, C, out_dtype=dtype)
        assert np.array_equal(got, want), (case["name"], alpha, beta, info)
        # uniform operands: within the summation error bound
        A, B, C = _inputs(case, dtype, 11, integer=False)
        got, _ = _run(case, dtype, A, B, C, alpha, beta)
        exact = tc.contract(la, A, sa, lb, B, sb, lc, sc, alpha, beta, C, out_dtype=F64)
        err = np.abs(got.astype(np.float64) - exact)
        assert np.all(err <= _bound(case, dtype, A, B, C, alpha, beta)), (case["name"], float(err.max()))


def test_beta_zero_never_reads_c_and_workspace_contents_do_not_matter():
    case = next(c for c in workloads.CONTRACTION_PARITY if c["name"] == "4d_reordered")
    sa, sb, sc = workloads.contraction_sizes(case)
    A, B, _ = _inputs(case, F32, 5, integer=True)
    C = np.full(int(np.prod(sc)), np.nan, dtype=F32)
    got, _ = _run(case, F32, A, B, C, 2.0, 0.0, pad_ws=1)   # workspace off 256-B alignment, filled with NaN
    want = tc.contract(case["labels_a"], A, sa, case["labels_b"], B, sb, case["labels_c"], sc, 2.0)
    assert np.array_equal(got, want)


def test_repeated_calls_share_one_workspace():
    """Two contractions of different shapes, one after the other on one
    workspace (sized for the larger), each equal to the oracle."""
    import torch
    cases = [c for c in workloads.CONTRACTION_PARITY if c["name"] in ("6d_result", "k_order_differs")]
    plans = []
    try:
        for c in cases:
            sa, sb, sc = workloads.contraction_sizes(c)
            plans.append(ttx.ttx_contraction_create(ttx.F32, c["labels_a"], sa, c["labels_b"], sb, c["labels_c"],
                                                    sc))
        ws_bytes = max(ttx.ttx_contraction_describe(p)["workspace_bytes"] for p in plans)
        ws = torch.empty(ws_bytes // 4 + 64, dtype=torch.float32, device="cuda")
        outs = []
        for c, p in zip(cases, plans):
            A, B, C = _inputs(c, F32, 8, integer=True)
            dA, pa = to_device(A)
            dB, pb = to_device(B)
            dC, pc = to_device(C)
            ttx.ttx_contraction_execute(p, 1.0, pa, pb, 1.0, pc, ws.data_ptr(), ttx.current_stream())
            outs.append((c, A, B, C, dC, dA, dB))
        for c, A, B, C, dC, dA, dB in outs:
            sa, sb, sc = workloads.contraction_sizes(c)
            want = tc.contract(c["labels_a"], A, sa, c["labels_b"], B, sb, c["labels_c"], sc, 1.0, 1.0, C)
            assert np.array_equal(from_device(dC), want), c["name"]
    finally:
        for p in plans:
            ttx.ttx_contraction_destroy(p)


@pytest.mark.parametrize("case", workloads.CONTRACTIONS, ids=lambda c: c["name"])
def test_full_size_sampled(case):
    """The measured contractions at full size: 256 sampled C elements (the
    first and last among them) against the oracle element by element, within
    the summation error bound."""
    dtype = np.dtype(case["dtype"])
    sa, sb, sc = workloads.contraction_sizes(case)
    la, lb, lc = case["labels_a"], case["labels_b"], case["labels_c"]
    A, B, C = _inputs(case, dtype, 21, integer=False)
    _say("%s: C %.0f MiB" % (case["name"], C.nbytes / 2 ** 20))
    got, info = _run(case, dtype, A, B, C, case["alpha"], case["beta"])
    rng = np.random.default_rng(22)
    pos = np.unique(np.concatenate([[0, C.size - 1], rng.integers(0, C.size, 254)]))
    exact = tc.contract_at(la, A, sa, lb, B, sb, lc, sc, pos, case["alpha"], case["beta"], C, out_dtype=F64)
    k = info["k"]
    mag = tc.contract_at(la, np.abs(A), sa, lb, np.abs(B), sb, lc, sc, pos, out_dtype=F64)
    bound = (k + 4) * UNIT[dtype] * (abs(case["alpha"]) * mag + abs(case["beta"]) * np.abs(C[pos].astype(F64)))
    err = np.abs(got[pos].astype(F64) - exact)
    assert np.all(err <= bound), (case["name"], float(err.max()))
    assert np.isfinite(got).all()
