"""GPU parity at full size (about 200 MiB per tensor) for the complex and
mixed-precision cases of the throughput run, as it runs them: the shipped
tune table loaded, each case through a plan with its size-specialised
kernel (the table's configuration for specialised execution where it has
one, with its workgroup size and LDS padding), the whole B compared with
the oracle element by element (at most 1 ulp per part; bit-identity is
expected and the count of differing elements is reported)."""
import os
import sys

import numpy as np
import pytest

import oracle
import paper_1607_01249_amd as ttx
import workloads
from gpu_util import assert_parity, dtype_code, from_device, to_device

pytestmark = pytest.mark.gpu

TABLE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                     "paper_1607_01249_amd", "tune", "gfx950.txt")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def shipped_table():
    ttx.ttx_tune_table_clear()
    ttx.ttx_tune_table_load(TABLE)
    yield
    ttx.ttx_tune_table_clear()


@pytest.mark.parametrize("case", workloads.complex_cases() + workloads.mixed_cases(), ids=lambda c: c["name"])
def test_full_size_specialised_types(case, shipped_table):
    perm, size = case["perm"], case["size"]
    code = dtype_code(case["dtype_a"], case["dtype"])
    n = workloads.elements(size)
    A = workloads.uniform(n, case["dtype_a"], case["seed_a"])
    B = workloads.uniform(n, case["dtype"], case["seed_b"])
    ref = B.copy()
    assert oracle.transpose(perm, size, case["alpha"], A, case["beta"], ref) == 0
    dA, pa = to_device(A)
    dB, pb = to_device(B)
    plan = ttx.ttx_plan_create(code, perm, size)
    try:
        assert ttx.ttx_plan_describe(plan)["config_from_table"][0], "case missing from the shipped table"
        assert ttx.ttx_plan_specialise(plan, False)
        kernel = ttx.ttx_plan_kernel_name(plan, 1.0, pa, pb)
        assert kernel.startswith("ttx_jit_"), kernel
        _say("%s: %s" % (case["name"], kernel))
        ttx.ttx_plan_execute_c(plan, case["alpha"], pa, case["beta"], pb, pb, ttx.current_stream())
    finally:
        ttx.ttx_plan_destroy(plan)
    assert_parity(from_device(dB), ref, exact=False, what=case["name"])
    del dA, dB
