"""Host-side checks of the contraction plan (no GPU): the index groups and
orders it picks, which operands it transposes, the packing kinds, the
workspace size, and argument errors (raised before any device work, so
fake device addresses are enough)."""
import numpy as np
import pytest

import paper_1607_01249_amd as ttx
import workloads


def _plan(case, dtype=ttx.F32):
    sa, sb, sc = workloads.contraction_sizes(case)
    p = ttx.ttx_contraction_create(dtype, case["labels_a"], sa, case["labels_b"], sb, case["labels_c"], sc)
    try:
        return ttx.ttx_contraction_describe(p)
    finally:
        ttx.ttx_contraction_destroy(p)


def _case(name):
    return next(c for c in workloads.CONTRACTION_PARITY + workloads.CONTRACTIONS if c["name"] == name)


def test_matrix_operands_are_packed_as_stored():
    d = _plan(_case("matrix_product"))
    assert (d["m"], d["n"], d["k"]) == (70, 45, 33)
    assert not d["transposed_a"] and not d["transposed_b"]
    assert (d["pack_kind_a"], d["pack_kind_b"]) == (ttx.PACK_MFMA_A, ttx.PACK_MFMA_B)
    # A stored k-major and B stored n-major: the other panel kind reads each as stored
    d = _plan(_case("k_major_operands"))
    assert not d["transposed_a"] and not d["transposed_b"]
    assert (d["pack_kind_a"], d["pack_kind_b"]) == (ttx.PACK_MFMA_B, ttx.PACK_MFMA_A)


def test_groups_and_orders():
    d = _plan(_case("4d_reordered"))
    assert d["order_m"] == [2, 0] and d["order_n"] == [3, 1] and d["order_k"] == [4, 5]
    assert d["transposed_a"] and d["transposed_b"]
    assert (d["m"], d["n"], d["k"]) == (45, 42, 44)
    d = _plan(_case("outer_product"))
    assert d["k"] == 1 and d["order_k"] == [] and not d["transposed_a"] and not d["transposed_b"]
    d = _plan(_case("inner_product"))   # contracted orders differ: one operand is transposed
    assert (d["m"], d["n"], d["k"]) == (1, 1, 31 * 29)
    assert d["transposed_a"] != d["transposed_b"]


def test_one_operand_already_a_matrix():
    """A is (M, K) as stored; B's contracted labels are in another order
    and it is transposed into A's."""
    case = dict(labels_a=(0, 1, 2, 3), labels_b=(3, 4, 2), labels_c=(0, 1, 4),
                extent={0: 3, 1: 4, 2: 5, 3: 6, 4: 7})
    d = _plan(case)
    assert not d["transposed_a"] and d["transposed_b"] and d["order_k"] == [2, 3]


def test_workspace_size():
    d = _plan(_case("4d_reordered"), ttx.F64)
    m, n, k, panel = d["m"], d["n"], d["k"], d["panel"]
    assert panel == 16
    kb = 64 // panel
    K = -(-k // kb) * kb
    up = lambda b: -(-b // 256) * 256
    want = up(m * k * 8) + up(k * n * 8) + up(-(-m // panel) * panel * K * 8) + up(-(-n // panel) * panel * K * 8) \
        + up(m * n * 8)
    assert d["workspace_bytes"] == want
    assert _plan(_case("empty_free"))["workspace_bytes"] == 0


def test_panel_choice():
    assert _plan(_case("matrix_product"))["panel"] == 32
    assert _plan(_case("matrix_product"), ttx.F64)["panel"] == 16
    assert _plan(_case("matrix_vector"))["panel"] == 16


@pytest.mark.parametrize("bad,status", [
    (((0, 0), (2, 2), (0, 1), (2, 3), (1,), (3,)), ttx.EINVAL),
    (((0, 1), (2, 2), (1, 2), (3, 3), (0, 2), (2, 3)), ttx.EINVAL),
    (((0, 1, 3), (2, 2, 2), (1, 2, 3), (2, 3, 2), (0, 2, 3), (2, 3, 2)), ttx.EINVAL),
    (((0, 1, 4), (2, 2, 2), (1, 2), (2, 3), (0, 2), (2, 3)), ttx.EINVAL),
    (((0, 1), (2, -1), (1, 2), (-1, 3), (0, 2), (2, 3)), ttx.EINVAL),
])
def test_label_errors(bad, status):
    with pytest.raises(ttx.TTXError) as e:
        ttx.ttx_contraction_create(ttx.F32, *bad)
    assert e.value.status == status


def test_unsupported_types():
    for code in (ttx.C32, ttx.C64, ttx.CODE_OF[(ttx.F32, ttx.F64)]):
        with pytest.raises(ttx.TTXError) as e:
            ttx.ttx_contraction_create(code, (0, 2), (4, 5), (2, 1), (5, 6), (0, 1), (4, 6))
        assert e.value.status == ttx.EUNSUPPORTED


def test_execute_argument_errors_before_device_work():
    p = ttx.ttx_contraction_create(ttx.F32, (0, 2), (64, 32), (2, 1), (32, 48), (0, 1), (64, 48))
    try:
        ws = ttx.ttx_contraction_describe(p)["workspace_bytes"]
        A, B, C, W = 1 << 32, 1 << 33, 1 << 34, 1 << 35
        cases = [
            ((A, B, C, 0), ttx.EINVAL),                 # no workspace
            ((A, B, 0, W), ttx.EINVAL),                 # no C
            ((A + 2, B, C, W), ttx.EINVAL),             # misaligned
            ((A, B, A + 64, W), ttx.EOVERLAP),          # C inside A
            ((A, B, C, C + 4 * 64 * 48 - 4), ttx.EOVERLAP),   # workspace starts in C's last element
            ((A, B, C, B - ws + 4), ttx.EOVERLAP),      # workspace ends in B's first element
        ]
        for (a, b, c, w), status in cases:
            with pytest.raises(ttx.TTXError) as e:
                ttx.ttx_contraction_execute(p, 1.0, a, b, 0.0, c, w)
            assert e.value.status == status, (a, b, c, w)
    finally:
        ttx.ttx_contraction_destroy(p)


def test_empty_result_launches_nothing():
    """m * n == 0: C has no elements; execution returns before touching any pointer."""
    case = _case("empty_free")
    sa, sb, sc = workloads.contraction_sizes(case)
    p = ttx.ttx_contraction_create(ttx.F32, case["labels_a"], sa, case["labels_b"], sb, case["labels_c"], sc)
    try:
        ttx.ttx_contraction_execute(p, 1.0, 0, 0, 0.0, 0, 0)
    finally:
        ttx.ttx_contraction_destroy(p)


def test_every_parity_case_plans():
    for case in workloads.CONTRACTION_PARITY + workloads.CONTRACTIONS:
        for dtype in (ttx.F32, ttx.F64):
            d = _plan(case, dtype)
            e = case["extent"]
            assert d["m"] == int(np.prod([e[l] for l in d["order_m"]], dtype=np.int64))
            assert d["n"] == int(np.prod([e[l] for l in d["order_n"]], dtype=np.int64))
            assert d["k"] == int(np.prod([e[l] for l in d["order_k"]], dtype=np.int64))
            assert sorted(d["order_m"] + d["order_n"]) == sorted(case["labels_c"])
