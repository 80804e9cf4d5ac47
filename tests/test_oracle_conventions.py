"""Pins for the oracle's index conventions and products (section 2.2):
brute-force index loops written from the definitions, and hand-derived
values under tests/golden/."""

import itertools
import json
import os

import numpy as np
import pytest

from oracle import tensor as T

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "conventions.json")))


def brute_kron(A, B):
    I, J = A.shape
    K, M = B.shape
    out = np.zeros((I * K, J * M))
    for i, j, k, l in itertools.product(range(I), range(J), range(K), range(M)):
        out[K * i + k, M * j + l] = A[i, j] * B[k, l]
    return out


def brute_unfold(X, n):
    shape = X.shape
    rest = [k for k in range(X.ndim) if k != n]
    ncol = int(np.prod([shape[k] for k in rest]))
    out = np.zeros((shape[n], ncol))
    for idx in itertools.product(*[range(s) for s in shape]):
        col, stride = 0, 1
        for k in rest:
            col += idx[k] * stride
            stride *= shape[k]
        out[idx[n], col] = X[idx]
    return out


def brute_ttm(X, U, n):
    shape = list(X.shape)
    oshape = shape.copy()
    oshape[n] = U.shape[0]
    Y = np.zeros(oshape)
    for idx in itertools.product(*[range(s) for s in oshape]):
        s = 0.0
        for i in range(shape[n]):
            src = list(idx)
            src[n] = i
            s += X[tuple(src)] * U[idx[n], i]
        Y[idx] = s
    return Y


def test_golden_kron_krp():
    g = GOLD["kron"]
    np.testing.assert_array_equal(T.kron(np.array(g["A"]), np.array(g["B"])), np.array(g["A_kron_B"]))
    g = GOLD["khatri_rao"]
    np.testing.assert_array_equal(T.khatri_rao(np.array(g["A"]), np.array(g["B"])), np.array(g["A_krp_B"]))


def test_golden_unfold_ttm():
    g = GOLD["unfold"]
    shape = tuple(g["shape"])
    X = np.zeros(shape)
    for i, j, k in itertools.product(*[range(s) for s in shape]):
        X[i, j, k] = (i + 1) + 3 * j + 12 * k
    for n, key in enumerate(["X1", "X2", "X3"]):
        np.testing.assert_array_equal(T.unfold(X, n), np.array(g[key]))
        np.testing.assert_array_equal(T.fold(T.unfold(X, n), n, shape), X)
    U = np.array(GOLD["ttm"]["U"], dtype=float)
    np.testing.assert_array_equal(T.unfold(T.ttm(X, U, 1), 1), np.array(GOLD["ttm"]["Y2"]))


@pytest.mark.parametrize("shapes", [((3, 4), (2, 5)), ((1, 3), (4, 1)), ((2, 2), (3, 3))])
def test_kron_brute(shapes):
    rng = np.random.default_rng(1)
    A = rng.standard_normal(shapes[0])
    B = rng.standard_normal(shapes[1])
    np.testing.assert_array_equal(T.kron(A, B), brute_kron(A, B))


def test_khatri_rao_brute():
    rng = np.random.default_rng(2)
    A, B, C = rng.standard_normal((3, 4)), rng.standard_normal((5, 4)), rng.standard_normal((2, 4))
    KR = T.khatri_rao_list([A, B, C])
    for k in range(4):
        np.testing.assert_allclose(KR[:, k], brute_kron(brute_kron(A[:, [k]], B[:, [k]]), C[:, [k]])[:, 0],
                                   rtol=0, atol=1e-15)


@pytest.mark.parametrize("shape", [(3, 4, 5), (2, 3, 2, 3), (2, 1, 3, 2, 2)])
def test_unfold_ttm_brute(shape):
    rng = np.random.default_rng(3)
    X = rng.standard_normal(shape)
    for n in range(len(shape)):
        np.testing.assert_array_equal(T.unfold(X, n), brute_unfold(X, n))
        U = rng.standard_normal((3, shape[n]))
        np.testing.assert_allclose(T.ttm(X, U, n), brute_ttm(X, U, n), rtol=0, atol=1e-13)


def test_full_brute():
    rng = np.random.default_rng(4)
    shape, R = (3, 4, 2, 3), 3
    A = [rng.standard_normal((s, R)) for s in shape]
    lam = rng.random(R) + 0.5
    Xh = T.full(lam, A)
    for idx in itertools.product(*[range(s) for s in shape]):
        v = sum(lam[r] * np.prod([A[k][idx[k], r] for k in range(4)]) for r in range(R))
        assert abs(Xh[idx] - v) < 1e-13


def test_kr_identity():
    """eq. (kr-id): (C kron D)(A (.) B) = (CA) (.) (DB) whenever the products
    are defined and A, B have the same column count."""
    rng = np.random.default_rng(5)
    A, B = rng.standard_normal((4, 6)), rng.standard_normal((3, 6))
    C, D = rng.standard_normal((5, 4)), rng.standard_normal((2, 3))
    lhs = T.kron(C, D) @ T.khatri_rao(A, B)
    rhs = T.khatri_rao(C @ A, D @ B)
    np.testing.assert_allclose(lhs, rhs, rtol=0, atol=1e-13)


def test_multittm_kron_form_and_order():
    """eq. (multittm): Y_(n) = X_(n) (U_N kron ... kron U_1)^T skipping n, and
    any TTM order gives the same tensor (section 2.2)."""
    rng = np.random.default_rng(6)
    for shape in [(4, 3, 5), (3, 4, 2, 3), (2, 3, 2, 2, 3)]:
        N = len(shape)
        U = [rng.standard_normal((2, s)) for s in shape]
        for n in range(N):
            K = T.kron_list([U[k] for k in reversed(range(N)) if k != n])
            X = rng.standard_normal(shape)
            ref = T.unfold(X, n) @ K.T
            for order in itertools.permutations([k for k in range(N) if k != n]):
                Y = T.multittm(X, U, n, order=list(order))
                np.testing.assert_allclose(T.unfold(Y, n), ref, rtol=0, atol=1e-12)


def test_multittm_brute_sum():
    """Multi-TTM entry = sum over contracted indices of X times the U entries."""
    rng = np.random.default_rng(7)
    shape = (3, 2, 4)
    X = rng.standard_normal(shape)
    U = [rng.standard_normal((2, s)) for s in shape]
    Y = T.multittm(X, U, 1)
    for a, i, c in itertools.product(range(2), range(2), range(2)):
        v = sum(X[p, i, q] * U[0][a, p] * U[2][c, q] for p in range(3) for q in range(4))
        assert abs(Y[a, i, c] - v) < 1e-13


def test_mttkrp_brute():
    rng = np.random.default_rng(8)
    shape, R = (3, 4, 2), 3
    X = rng.standard_normal(shape)
    A = [rng.standard_normal((s, R)) for s in shape]
    for n in range(3):
        M = T.mttkrp(X, A, n)
        for i in range(shape[n]):
            for r in range(R):
                v = 0.0
                for idx in itertools.product(*[range(s) for s in shape]):
                    if idx[n] != i:
                        continue
                    v += X[idx] * np.prod([A[k][idx[k], r] for k in range(3) if k != n])
                assert abs(M[i, r] - v) < 1e-13
