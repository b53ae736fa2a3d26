"""Error model of the split-BF16 contractions, emulated exactly in numpy: each
FP32 operand is split by truncation into bfloat16 terms (hi, [mid,] lo) and
the products two levels below the leading one are dropped.  The bounds here
are the per-product errors the reduced-precision tolerances are built on:
hi/lo keeps about 15-16 bits of each operand and about 13 bits of each
product; hi/mid/lo keeps each FP32 operand exactly and each product to about
21 bits (FP32 rounding is 24)."""
import numpy as np
import pytest


def _split(a, ns):
    r = a.astype(np.float32)
    terms = []
    for _ in range(ns):
        h = (r.view(np.uint32) & np.uint32(0xFFFF0000)).view(np.float32)
        terms.append(h.astype(np.float64))
        r = (r - h).astype(np.float32)     # exact: h holds the leading bits of r
    return terms


def _kept(A, B):
    if len(A) == 2:
        return A[0] * B[0] + A[0] * B[1] + A[1] * B[0]
    return A[0] * B[0] + A[0] * B[1] + A[1] * B[0] + A[0] * B[2] + A[1] * B[1] + A[2] * B[0]


@pytest.mark.parametrize("ns,op_bound,prod_bound", [(2, 2.0 ** -15, 2.0 ** -13), (3, 0.0, 2.0 ** -21)])
def test_split_operand_and_product_error(ns, op_bound, prod_bound):
    rng = np.random.default_rng(ns)
    # magnitudes over many binades, both signs
    a = (rng.standard_normal(200_000) * 2.0 ** rng.integers(-20, 20, 200_000)).astype(np.float32)
    b = (rng.standard_normal(200_000) * 2.0 ** rng.integers(-20, 20, 200_000)).astype(np.float32)
    A, B = _split(a, ns), _split(b, ns)
    for t in A:  # every term is a bfloat16 value
        assert np.all((t.astype(np.float32).view(np.uint32) & 0xFFFF) == 0)
    op_err = np.abs(sum(A) - a.astype(np.float64)) / np.abs(a.astype(np.float64))
    assert op_err.max() <= op_bound
    exact = a.astype(np.float64) * b.astype(np.float64)
    prod_err = np.abs(_kept(A, B) - exact) / np.abs(exact)
    assert prod_err.max() <= prod_bound
    # the bound is not loose by more than a factor of 8
    assert prod_err.max() > prod_bound / 8
