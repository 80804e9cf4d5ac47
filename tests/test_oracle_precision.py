"""Pins for the reduced-precision emulation in oracle/precision.py: bit-level
bfloat16 rounding against PyTorch's own float32 -> bfloat16 conversion
(round to nearest, ties to even), the algebra of the hi/lo split, and the
error of the split and plain contractions against their bounds."""

import numpy as np
import pytest
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


def _bf16_lib(a):
    """bfloat16 rounding by PyTorch's own conversion (independent of the
    oracle's bit manipulation)."""
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(torch.bfloat16).to(torch.float32).numpy()


def explicit_lowp(X, Qs, n, mode):
    """The reduced-precision Multi-TTM written out product by product: for
    each TTM (decreasing mode size, ties by ascending mode), every entry of
    the new FP32 intermediate is the correctly rounded sum (math.fsum) of the
    kept partial products of bfloat16 operands -- x_hi q_hi (+ x_hi q_lo +
    x_lo q_hi for the split form), with x_lo = bf16(x - x_hi) taken in FP32 --
    rounded once to FP32.  Returns Y_(n) with column index sum_k r_k R^j over
    the modes k != n in increasing order (r of the lowest mode fastest)."""
    import itertools
    import math
    N = X.ndim
    order = sorted((k for k in range(N) if k != n), key=lambda k: (-X.shape[k], k))
    Tt = np.array(X, dtype=np.float32)
    for k in order:
        Q32 = np.asarray(Qs[k], dtype=np.float32)
        qh = _bf16_lib(Q32)
        ql = _bf16_lib((Q32 - qh).astype(np.float32))
        th = _bf16_lib(Tt)
        tl = _bf16_lib((Tt - th).astype(np.float32))
        R = Q32.shape[1]
        shape = list(Tt.shape)
        shape[k] = R
        out = np.empty(shape, dtype=np.float32)
        for idx in itertools.product(*[range(s) for s in shape]):
            r = idx[k]
            terms = []
            for i in range(Tt.shape[k]):
                src = idx[:k] + (i,) + idx[k + 1:]
                terms.append(float(th[src]) * float(qh[i, r]))
                if mode == "bf16x2":
                    terms.append(float(th[src]) * float(ql[i, r]))
                    terms.append(float(tl[src]) * float(qh[i, r]))
            out[idx] = np.float32(math.fsum(terms))
        Tt = out
    R = np.asarray(Qs[order[0]]).shape[1]
    others = [k for k in range(N) if k != n]
    Y = np.empty((X.shape[n], R ** (N - 1)), dtype=np.float64)
    for idx in itertools.product(*[range(s) for s in Tt.shape]):
        col = sum(idx[k] * R ** j for j, k in enumerate(others))
        Y[idx[n], col] = float(Tt[idx])
    return Y


@pytest.mark.parametrize("shape,R", [((5, 4, 6), 3), ((3, 4, 3, 2), 2)])
@pytest.mark.parametrize("mode", ["bf16", "bf16x2"])
def test_multittm_lowp_against_explicit_products(shape, R, mode):
    """On data that is not bfloat16-exact (Gaussian values with full FP32
    mantissas, so x_lo != 0 and every intermediate rounds), the emulation
    equals the product-by-product definition bit for bit: operands split or
    rounded as the form states, the x_lo q_lo term dropped, each TTM's result
    stored in FP32 before the next split."""
    rng = np.random.default_rng(sum(shape) * 7 + R)
    X = rng.standard_normal(shape).astype(np.float32)
    Qs = [rng.standard_normal((s, R)) for s in shape]
    assert np.any(P.split_bf16(X)[1] != 0)
    for n in range(len(shape)):
        want = explicit_lowp(X, Qs, n, mode)
        got = P.multittm_lowp(X, Qs, n, mode)
        assert np.array_equal(got, want), (n, np.abs(got - want).max())


def test_planted_split_dispatch_is_caught(monkeypatch):
    """Taking the plain form where the split one is asked for is caught."""
    rng = np.random.default_rng(9)
    X = rng.standard_normal((5, 4, 6)).astype(np.float32)
    Qs = [rng.standard_normal((s, 3)) for s in X.shape]
    want = explicit_lowp(X, Qs, 0, "bf16x2")
    monkeypatch.setattr(P, "contract_split", P.contract_bf16)
    assert not np.array_equal(P.multittm_lowp(X, Qs, 0, "bf16x2"), want)


def test_planted_missing_fp32_store_is_caught(monkeypatch):
    """An emulation that kept its final intermediate in FP64 (no FP32 store)
    differs from the definition in most entries (split products carry more
    bits than FP32 holds)."""
    from oracle import tensor as OT2
    rng = np.random.default_rng(10)
    X = rng.standard_normal((5, 4, 6)).astype(np.float32)
    Qs = [rng.standard_normal((s, 3)) for s in X.shape]
    want = explicit_lowp(X, Qs, 1, "bf16x2")

    def no_store(X, Qs, n, mode, order=None):
        if order is None:
            order = OT2.multittm_order(X.shape, n)
        Y = np.asarray(X, dtype=np.float32)
        for k in order:
            Q = np.asarray(Qs[k], dtype=np.float64)
            Z = P.contract_split(OT2.unfold(Y, k).T.astype(np.float32), Q.astype(np.float32))
            shape = list(Y.shape)
            shape[k] = Q.shape[1]
            Y = OT2.fold(Z.T, k, shape)
        return OT2.unfold(Y, n).astype(np.float64)
    got = no_store(X, Qs, 1, "bf16x2")
    assert np.mean(got != want) > 0.5
