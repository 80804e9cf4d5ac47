"""Pins for the reduced-precision emulation in oracle/precision.py: bit-level
bfloat16 rounding against PyTorch's own float32 -> bfloat16 conversion
(round to nearest, ties to even), the algebra of the hi/lo split, and the
error of the split and plain contractions against their bounds."""

import numpy as np
import torch

from oracle import precision as P
from oracle import tensor as T
import oracle.cp_als_qr as OQ


def test_round_bf16_matches_library_rounding():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(20000).astype(np.float32) * 10.0 ** rng.integers(-30, 30, 20000),
                        np.array([0.0, -0.0, 1.0, -1.0, 3.0e38, 1e-40, np.inf, -np.inf], dtype=np.float32)])
    # ties: values exactly half-way between two bfloat16 numbers
    ties = (np.arange(1, 200, dtype=np.uint32) << 16) | 0x8000
    x = np.concatenate([x, ties.view(np.float32)])
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    got = P.round_bf16(x)
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))


def test_split_algebra():
    rng = np.random.default_rng(1)
    x = rng.standard_normal(10000).astype(np.float32)
    hi, lo = P.split_bf16(x)
    assert np.array_equal(P.round_bf16(hi), hi) and np.array_equal(P.round_bf16(lo), lo)
    # hi carries 8 significant bits, lo the next 8: |x - hi - lo| <= 2^-16 |x| (plus rounding of lo)
    err = np.abs(x.astype(np.float64) - hi - lo)
    assert np.all(err <= 2.0 ** -16 * np.abs(x) + 1e-45)


def test_contraction_error_bounds():
    rng = np.random.default_rng(2)
    A = rng.standard_normal((200, 300)).astype(np.float32)
    B = rng.standard_normal((300, 16)).astype(np.float32)
    exact = A.astype(np.float64) @ B.astype(np.float64)
    bound = np.abs(A.astype(np.float64)) @ np.abs(B.astype(np.float64))
    e_split = np.abs(P.contract_split(A, B) - exact)
    e_bf16 = np.abs(P.contract_bf16(A, B) - exact)
    # three kept products: per product error <= 3 * 2^-16 + 2^-32 relative
    assert np.all(e_split <= 3.1 * 2.0 ** -16 * bound)
    # plain bf16: per product error <= 2 * 2^-9 relative
    assert np.all(e_bf16 <= 2.1 * 2.0 ** -9 * bound)
    # and the split form is at least 100x more accurate than plain bf16
    assert np.linalg.norm(e_split) < 1e-2 * np.linalg.norm(e_bf16)


def test_multittm_lowp_reduces_to_exact_on_representable_data():
    """With data and operands exactly representable in bfloat16 and small
    integer values (exact sums), every form equals the exact Multi-TTM."""
    rng = np.random.default_rng(3)
    shape = (6, 5, 4)
    X = rng.integers(-8, 8, shape).astype(np.float32)
    Qs = [rng.integers(-4, 4, (s, 3)).astype(np.float64) for s in shape]
    for n in range(3):
        ref = T.unfold(T.multittm(X.astype(np.float64), [q.T for q in Qs], n), n)
        for mode in ("bf16", "bf16x2"):
            np.testing.assert_array_equal(P.multittm_lowp(X, Qs, n, mode), ref)
