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


def _random_contraction(rng):
    """Random labels: up to 3 free labels per operand and 3 contracted, shuffled per tensor."""
    nm, nn, nk = (int(x) for x in rng.integers(0, 4, 3))
    labels = list(rng.permutation(20)[:nm + nn + nk])
    M, N, K = labels[:nm], labels[nm:nm + nn], labels[nm + nn:]
    ext = {l: int(rng.integers(1, 5)) for l in labels}
    la = list(rng.permutation(M + K)) if rng.random() < 0.6 else M + K   # often already a matrix
    lb = list(rng.permutation(K + N)) if rng.random() < 0.6 else (K + N if rng.random() < 0.5 else N + K)
    lc = list(rng.permutation(M + N))
    return [int(x) for x in la], [int(x) for x in lb], [int(x) for x in lc], ext


def test_random_plans_are_consistent_and_replay_to_the_oracle():
    """For 300 random contractions: the plan's index groups are A's free,
    B's free and the contracted labels; an operand left untransposed is
    stored as its two blocks in the order its pack kind reads; and replaying
    the planned steps on the CPU (operands into the planned orders, matrix
    product, product into C's order) gives the oracle's result."""
    from oracle import tensor_contract as tc
    rng = np.random.default_rng(77)
    for _ in range(300):
        la, lb, lc, ext = _random_contraction(rng)
        sa, sb, sc = ([ext[l] for l in ls] for ls in (la, lb, lc))
        p = ttx.ttx_contraction_create(ttx.F64, la, sa, lb, sb, lc, sc)
        try:
            d = ttx.ttx_contraction_describe(p)
        finally:
            ttx.ttx_contraction_destroy(p)
        om, on, ok = d["order_m"], d["order_n"], d["order_k"]
        assert sorted(om) == sorted(l for l in la if l in lc)
        assert sorted(on) == sorted(l for l in lb if l in lc)
        assert sorted(ok) == sorted(l for l in la if l in lb)
        prod = lambda ls: int(np.prod([ext[l] for l in ls], dtype=np.int64))
        assert (d["m"], d["n"], d["k"]) == (prod(om), prod(on), prod(ok))
        if not d["transposed_a"]:
            assert la == (om + ok if d["pack_kind_a"] == ttx.PACK_MFMA_A else ok + om), (la, d)
        if not d["transposed_b"]:
            assert lb == (ok + on if d["pack_kind_b"] == ttx.PACK_MFMA_B else on + ok), (lb, d)
        A = rng.standard_normal(prod(la))
        B = rng.standard_normal(prod(lb))
        # replay: column-major tensors as numpy arrays indexed in label order
        a = A.reshape([ext[l] for l in la], order="F") if la else A.reshape(())
        b = B.reshape([ext[l] for l in lb], order="F") if lb else B.reshape(())
        am = np.transpose(a, [la.index(l) for l in om + ok]).reshape((d["m"], d["k"]), order="F")
        bm = np.transpose(b, [lb.index(l) for l in ok + on]).reshape((d["k"], d["n"]), order="F")
        cm = (am @ bm).reshape([ext[l] for l in om + on] or [1], order="F")
        got = np.transpose(cm.reshape([ext[l] for l in om + on]) if om + on else cm.reshape(()),
                           [(om + on).index(l) for l in lc]).reshape(-1, order="F")
        want = tc.contract(la, A, sa, lb, B, sb, lc, sc)
        np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-12)
