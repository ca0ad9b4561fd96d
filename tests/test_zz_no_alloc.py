"""GPU check of the allocation-free batched run (ttx_batch_run_static).

Two calls in a row through the C ABI, the second with fewer and smaller
problems than the first, so that it runs over what the first left in the
static work block: each must give the same bits as ttx_batch_create +
ttx_batch_execute on the same problems and inputs, and as the oracle.
"""
import sys

import numpy as np
import pytest

import oracle
import paper_1607_01249_amd as ttx
import workloads
from gpu_util import F32, assert_parity

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


class _Set:
    """Host inputs, device A and two device B copies (one per entry point)."""

    def __init__(self, probs, seed):
        import torch
        self.probs = probs
        self.A, self.B0, self.dA, self.dB = [], [], [], []
        for i, p in enumerate(probs):
            n = workloads.elements(p["size"])
            self.A.append(workloads.uniform(n, p["dtype"], seed + 2 * i))
            self.B0.append(workloads.uniform(n, p["dtype"], seed + 2 * i + 1))
            self.dA.append(torch.from_numpy(self.A[-1]).cuda())
            self.dB.append(torch.from_numpy(self.B0[-1]).cuda())
        torch.cuda.synchronize()

    def reset_b(self):
        import torch
        for d, b in zip(self.dB, self.B0):
            d.copy_(torch.from_numpy(b))
        torch.cuda.synchronize()

    def problems(self):
        return [ttx.make_problem(ttx.F32 if p["dtype"].itemsize == 4 else ttx.F64, p["perm"], p["size"],
                                 p["alpha"], a.data_ptr(), p["beta"], b.data_ptr())
                for p, a, b in zip(self.probs, self.dA, self.dB)]

    def results(self):
        import torch
        torch.cuda.synchronize()
        return [d.cpu().numpy() for d in self.dB]


def _bits_equal(xs, ys):
    bad = [i for i, (x, y) in enumerate(zip(xs, ys)) if not np.array_equal(x.view(np.uint8), y.view(np.uint8))]
    return bad


def _degenerate():
    f64 = np.dtype(np.float64)
    return [dict(dtype=F32, size=(0, 5), perm=(1, 0), alpha=1.0, beta=0.0),
            dict(dtype=F32, size=(1, 1, 1), perm=(2, 0, 1), alpha=2.0, beta=0.5),
            dict(dtype=f64, size=(7, 1, 9), perm=(0, 1, 2), alpha=-1.0, beta=0.25),
            dict(dtype=F32, size=(1000, 3), perm=(1, 0), alpha=1.0, beta=0.0)]


@pytest.mark.parametrize("call,count,seed,max_elems", [(1, 300, 31, 1 << 20), (2, 40, 32, 1 << 16)])
def test_static_run_matches_batch_execute(call, count, seed, max_elems):
    probs = workloads.batched_problems(count=count, seed=seed, max_elems=max_elems)
    if call == 1:
        probs = probs + _degenerate()
    _say("static batch call %d: %d problems, seed %d" % (call, len(probs), seed))
    s = _Set(probs, seed=1000 * call)
    stream = ttx.current_stream()
    # the existing entry point
    h = ttx.ttx_batch_create(s.problems())
    try:
        ttx.ttx_batch_execute(h, stream)
        want = s.results()
    finally:
        ttx.ttx_batch_destroy(h)
    # the allocation-free one, on the same inputs
    s.reset_b()
    ttx.ttx_batch_run_static(s.problems(), stream)
    got = s.results()
    bad = _bits_equal(got, want)
    assert not bad, "problems %s differ from ttx_batch_execute" % bad[:8]
    for i, (g, p, a, b) in enumerate(zip(got, probs, s.A, s.B0)):
        r = b.copy()
        assert oracle.transpose(p["perm"], p["size"], p["alpha"], a, p["beta"], r) == 0
        assert_parity(g, r, exact=(p["alpha"] == 1.0 and p["beta"] == 0.0), what="problem %d %s" % (i, p))


def test_static_run_refuses_too_many_problems():
    probs = [ttx.make_problem(ttx.F32, (1, 0), (2, 2), 1.0, 0, 0.0, 0)] * (ttx.STATIC_BATCH_MAX + 1)
    with pytest.raises(ttx.TTXError, match="at most"):
        ttx.ttx_batch_run_static(probs, ttx.current_stream())
