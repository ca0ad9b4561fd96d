"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module describes workloads only: shapes, permutations, scalars and
uniformly distributed element values drawn from numpy's PCG64 generator.
It holds none of the transposition's arithmetic; both the CPU oracle and the
HIP library receive exactly the bits produced here.

The paper's own benchmark (57 transpositions, 2D to 6D, about 200 MB per
tensor, Sec. 3) is not available; the shapes below stand in for it with the
same class of sizes.
"""
import math

import numpy as np

F32, F64 = np.dtype(np.float32), np.dtype(np.float64)
C32, C64 = np.dtype(np.complex64), np.dtype(np.complex128)


def uniform(n, dtype, seed):
    """n values uniform in [-1, 1) of the given dtype (exact on the dtype's grid);
    complex values have both parts drawn that way (real, imaginary, real, ...)."""
    dtype = np.dtype(dtype)
    if dtype in (C32, C64):
        parts = uniform(2 * int(n), F32 if dtype == C32 else F64, seed)
        return parts.view(dtype)
    rng = np.random.default_rng(seed)
    if dtype == F32:
        return rng.random(int(n), dtype=np.float32) * 2 - 1
    return rng.random(int(n)) * 2 - 1


def elements(size):
    return int(np.prod([int(s) for s in size], dtype=np.int64))


# -- plain single transposition (correctness case) ------------------------------------
PLAIN = dict(name="plain_3d_f32", dtype=F32, size=(96, 128, 80), perm=(2, 1, 0),
             alpha=1.0, beta=0.0, seed_a=0)

# -- paper-shaped large transpositions, about 200 MiB per tensor ----------------------
LARGE_SHAPES = {
    ("4d", F32): (160, 160, 64, 32),
    ("4d", F64): (160, 160, 32, 32),
    ("5d", F32): (40, 32, 40, 32, 32),
    ("5d", F64): (44, 32, 24, 32, 24),
    ("6d", F32): (24, 21, 20, 18, 17, 17),
    ("6d", F64): (20, 16, 16, 20, 16, 16),
}
LARGE_PERMS = {
    "4d": [(1, 0, 3, 2), (3, 2, 1, 0), (0, 2, 1, 3), (2, 0, 3, 1)],
    "5d": [(4, 3, 2, 1, 0), (1, 3, 0, 4, 2), (0, 3, 2, 4, 1)],
    "6d": [(5, 4, 3, 2, 1, 0), (0, 5, 1, 4, 2, 3)],
}
# the literal "(160,160,160,160)" shape: 2.44 GiB (FP32) / 4.88 GiB (FP64) per tensor
LITERAL_4D = (160, 160, 160, 160)
# the literal "all dims 24" 6D shape: 729 MiB (FP32) / 1458 MiB (FP64) per tensor
LITERAL_6D = (24, 24, 24, 24, 24, 24)


def large_cases(betas=(0.7, 0.0)):
    """All paper-shaped large cases: dicts with name, dtype, size, perm, alpha, beta, seeds."""
    out = []
    case = 0
    for rank in ("4d", "5d", "6d"):
        for dtype in (F32, F64):
            size = LARGE_SHAPES[(rank, dtype)]
            for perm in LARGE_PERMS[rank]:
                for beta in betas:
                    out.append(dict(
                        name="%s_%s_p%s_b%s" % (rank, "f32" if dtype == F32 else "f64",
                                                "".join(map(str, perm)), beta),
                        dtype=dtype, size=size, perm=perm, alpha=1.3, beta=beta,
                        seed_a=1000 + case, seed_b=2000 + case))
                    case += 1
    return out


# -- complex elements (the c and z types), about 200 MiB per tensor --------------------
# Single complex elements have the FP64 byte size and take the FP64 shapes;
# double complex halves the last extent.
COMPLEX_PERMS = {
    "4d": [(3, 2, 1, 0), (2, 0, 3, 1), (0, 2, 1, 3)],
    "5d": [(1, 3, 0, 4, 2), (0, 3, 2, 4, 1)],
    "6d": [(5, 4, 3, 2, 1, 0), (0, 5, 1, 4, 2, 3)],
}
COMPLEX_ALPHA, COMPLEX_BETA = complex(0.75, -1.25), complex(-0.5, 0.375)


def complex_shape(rank, dtype):
    size = list(LARGE_SHAPES[(rank, F64)])
    if np.dtype(dtype) == C64:
        size[-1] //= 2
    return tuple(size)


def complex_cases():
    """Large complex cases (complex alpha and beta, beta != 0); A and B of one type."""
    out = []
    case = 0
    for rank in ("4d", "5d", "6d"):
        for dtype in (C32, C64):
            for perm in COMPLEX_PERMS[rank]:
                out.append(dict(name="%s_%s_p%s" % (rank, "c32" if dtype == C32 else "c64",
                                                   "".join(map(str, perm))),
                                dtype_a=dtype, dtype=dtype, size=complex_shape(rank, dtype), perm=perm,
                                alpha=COMPLEX_ALPHA, beta=COMPLEX_BETA,
                                seed_a=5000 + case, seed_b=6000 + case))
                case += 1
    return out


# -- mixed precision (Table 1 "sd", "ds", "cz", "zc"): A's type, then B's -------------
MIXED_PAIRS = {"sd": (F32, F64), "ds": (F64, F32), "cz": (C32, C64), "zc": (C64, C32)}
MIXED_PERMS = [(3, 2, 1, 0), (2, 0, 3, 1), (0, 2, 1, 3)]


def mixed_cases():
    """Large 4D mixed-precision cases: the double (complex) side about 200 MiB."""
    out = []
    case = 0
    for name, (da, db) in MIXED_PAIRS.items():
        size = (160, 160, 32, 32) if da in (F32, F64) else (160, 160, 32, 16)
        cx = db in (C32, C64)
        for perm in MIXED_PERMS:
            out.append(dict(name="4d_%s_p%s" % (name, "".join(map(str, perm))), dtype_a=da, dtype=db,
                            size=size, perm=perm, alpha=COMPLEX_ALPHA if cx else 1.3,
                            beta=COMPLEX_BETA if cx else 0.7, seed_a=9000 + case, seed_b=9500 + case))
            case += 1
    return out


# -- multiple leading dimensions (BLAS-3 packing shapes) ------------------------------
LD_CASES = [
    dict(name="ld_f64_packing", dtype=F64, size=(384, 96, 48, 32), perm=(1, 0, 2, 3),
         outer_a=(400, 100, 48, 32), outer_b=(100, 400, 50, 32)),
    dict(name="awkward_f32", dtype=F32, size=(7, 1023, 33, 65), perm=(1, 2, 3, 0),
         outer_a=None, outer_b=None),
    dict(name="awkward_f64", dtype=F64, size=(7, 1023, 33, 65), perm=(1, 2, 3, 0),
         outer_a=None, outer_b=None),
]
LD_SCALARS = [(1.0, 0.0), (-0.5, 1.0)]


# -- batched: 512 uneven transpositions ----------------------------------------------
def batched_problems(count=512, seed=4, min_elems=4096, max_elems=4194304):
    """Random problems: N uniform in 2..6, random perm, element count log-uniform in
    [min_elems, max_elems] split across dims by a flat Dirichlet draw, 70% FP32,
    alpha uniform in [-2, 2], beta zero with probability 1/4 else uniform in [-2, 2].
    Degenerate draws (size-1 dims, identity after merging) are kept."""
    rng = np.random.default_rng(seed)
    probs = []
    for _ in range(count):
        n = int(rng.integers(2, 7))
        perm = tuple(int(p) for p in rng.permutation(n))
        e = math.exp(rng.uniform(math.log(min_elems), math.log(max_elems)))
        w = rng.dirichlet(np.ones(n))
        size = tuple(max(1, int(round(e ** float(wk)))) for wk in w)
        dtype = F32 if rng.random() < 0.7 else F64
        alpha = float(rng.uniform(-2, 2))
        beta = 0.0 if rng.random() < 0.25 else float(rng.uniform(-2, 2))
        probs.append(dict(dtype=dtype, size=size, perm=perm, alpha=alpha, beta=beta))
    return probs


# -- served: Poisson arrivals ---------------------------------------------------------
def served_trace(rate=20000.0, duration=10.0, seed_arrivals=5, seed_shapes=6,
                 large_frac=0.05, large_bytes=(64 << 20, 256 << 20)):
    """Open-loop request trace: arrival times (seconds, exponential gaps at ``rate``)
    and request shapes drawn as for the batched workload, with ``large_frac`` of
    requests large (bytes log-uniform in ``large_bytes``, N in 3..6)."""
    rng = np.random.default_rng(seed_arrivals)
    gaps = rng.exponential(1.0 / rate, size=int(rate * duration * 1.2) + 16)
    times = np.cumsum(gaps)
    times = times[times < duration]
    shapes = np.random.default_rng(seed_shapes)
    reqs = []
    for _ in range(len(times)):
        large = shapes.random() < large_frac
        n = int(shapes.integers(3, 7)) if large else int(shapes.integers(2, 7))
        perm = tuple(int(p) for p in shapes.permutation(n))
        dtype = F32 if shapes.random() < 0.7 else F64
        if large:
            nbytes = math.exp(shapes.uniform(math.log(large_bytes[0]), math.log(large_bytes[1])))
            e = nbytes / dtype.itemsize
        else:
            e = math.exp(shapes.uniform(math.log(4096), math.log(4194304)))
        w = shapes.dirichlet(np.ones(n))
        size = tuple(max(1, int(round(e ** float(wk)))) for wk in w)
        alpha = float(shapes.uniform(-2, 2))
        beta = 0.0 if shapes.random() < 0.25 else float(shapes.uniform(-2, 2))
        reqs.append(dict(dtype=dtype, size=size, perm=perm, alpha=alpha, beta=beta,
                         large=bool(large)))
    return times, reqs


# -- tensor contractions cast as transpose-transpose-GEMM-transpose ------------------------
# Binary contractions with integer mode labels (column-major tensors, labels in
# storage order); a label in A and B only is summed over.  The three measured
# ones span the two regimes of the approach: the matrix product dominates (all
# extents 40, m = n = k = 1600), or the transpositions do (small contracted
# extents, large free extents, where the operands' memory traffic is most of the
# work).  The parity cases add ragged panels, operands already in matrix order
# (no transposition), K-major operands, a scalar result and empty extents.
CONTRACTIONS = [
    dict(name="ttgt_gemm_bound_f32", dtype=F32, labels_a=(2, 4, 0, 5), labels_b=(5, 3, 4, 1),
         labels_c=(0, 1, 2, 3), extent={0: 40, 1: 40, 2: 40, 3: 40, 4: 40, 5: 40}, alpha=1.0, beta=0.0),
    dict(name="ttgt_small_k_f32", dtype=F32, labels_a=(2, 6, 0, 4), labels_b=(5, 3, 6, 1),
         labels_c=(0, 1, 2, 3, 4, 5), extent={0: 24, 1: 24, 2: 24, 3: 24, 4: 24, 5: 24, 6: 16}, alpha=1.0,
         beta=0.5),
    dict(name="ttgt_small_k_f64", dtype=F64, labels_a=(1, 3, 0), labels_b=(3, 2), labels_c=(0, 1, 2),
         extent={0: 96, 1: 64, 2: 512, 3: 8}, alpha=-1.5, beta=1.0),
]

CONTRACTION_PARITY = [  # small: the oracle contracts them whole in well under a second
    dict(name="matrix_product", labels_a=(0, 2), labels_b=(2, 1), labels_c=(0, 1), extent={0: 70, 1: 45, 2: 33}),
    dict(name="k_major_operands", labels_a=(2, 0), labels_b=(1, 2), labels_c=(0, 1), extent={0: 37, 1: 50, 2: 65}),
    dict(name="4d_reordered", labels_a=(2, 4, 0, 5), labels_b=(5, 3, 4, 1), labels_c=(0, 1, 2, 3),
         extent={0: 9, 1: 7, 2: 5, 3: 6, 4: 4, 5: 11}),
    dict(name="6d_result", labels_a=(2, 6, 0, 4), labels_b=(5, 3, 6, 1), labels_c=(0, 1, 2, 3, 4, 5),
         extent={0: 5, 1: 4, 2: 3, 3: 6, 4: 2, 5: 7, 6: 9}),
    dict(name="k_order_differs", labels_a=(0, 3, 4, 1), labels_b=(4, 2, 3), labels_c=(1, 2, 0),
         extent={0: 17, 1: 3, 2: 40, 3: 5, 4: 6}),
    dict(name="outer_product", labels_a=(1, 0), labels_b=(2,), labels_c=(0, 2, 1), extent={0: 33, 1: 3, 2: 20}),
    dict(name="inner_product", labels_a=(0, 1), labels_b=(1, 0), labels_c=(), extent={0: 31, 1: 29}),
    dict(name="matrix_vector", labels_a=(1, 0), labels_b=(1,), labels_c=(0,), extent={0: 100, 1: 77}),
    dict(name="empty_contracted", labels_a=(0, 2), labels_b=(2, 1), labels_c=(0, 1), extent={0: 8, 1: 9, 2: 0}),
    dict(name="empty_free", labels_a=(0, 2), labels_b=(2, 1), labels_c=(0, 1), extent={0: 0, 1: 9, 2: 5}),
    dict(name="scalars", labels_a=(), labels_b=(), labels_c=(), extent={}),
    dict(name="scalar_operand", labels_a=(1, 0), labels_b=(), labels_c=(0, 1), extent={0: 37, 1: 5}),
]


def contraction_sizes(case):
    """(size_a, size_b, size_c): the extents of each tensor's modes."""
    e = case["extent"]
    return tuple(tuple(e[l] for l in case[k]) for k in ("labels_a", "labels_b", "labels_c"))
