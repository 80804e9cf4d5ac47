"""Pins of oracle/learned.py to definitions it does not use itself:
brute-force index sums, dense reconstruction, central finite differences,
and Adam's closed-form first step.  Planted mistakes (in the oracle, on the
CPU) show that each pin can fail."""

import itertools

import numpy as np
import pytest

from oracle import learned as L
from oracle import tensor as T


def brute_sketch(X, S):
    I = X.shape
    J = [s.shape[0] for s in S]
    out = np.zeros(J)
    for j in itertools.product(*[range(n) for n in J]):
        acc = 0.0
        for i in itertools.product(*[range(n) for n in I]):
            acc += X[i] * S[0][j[0], i[0]] * S[1][j[1], i[1]] * S[2][j[2], i[2]]
        out[j] = acc
    return out


def test_sketch_equals_index_sum():
    rng = np.random.default_rng(3)
    X = rng.standard_normal((3, 4, 5))
    S = [rng.standard_normal((2, 3)), rng.standard_normal((3, 4)), rng.standard_normal((2, 5))]
    np.testing.assert_allclose(L.sketch(X, S), brute_sketch(X, S), rtol=1e-13, atol=1e-13)


def test_sketch_vector_order():
    Xs = np.arange(2 * 3 * 4, dtype=float).reshape(2, 3, 4)
    v = L.sketch_vector(Xs)
    for j1, j2, j3 in itertools.product(range(2), range(3), range(4)):
        assert v[j2 + 3 * j1 + 6 * j3] == Xs[j1, j2, j3]


def test_unpack_pack_roundtrip_and_layout():
    I, R = (3, 4, 2), 2
    y = np.arange(sum(I) * R, dtype=float)
    A = L.unpack_factors(y, I, R)
    assert A[0][1, 0] == 1.0 and A[0][0, 1] == 3.0  # column-major, first factor first
    assert A[1][0, 0] == 6.0
    np.testing.assert_array_equal(L.pack_factors(A), y)


def random_factors(rng, I, R):
    return [rng.standard_normal((n, R)) for n in I]


def test_kruskal_loss_equals_dense_reconstruction():
    rng = np.random.default_rng(5)
    I = (4, 5, 3)
    A = random_factors(rng, I, 3)
    Ah = random_factors(rng, I, 2)  # different ranks are allowed
    Xa = T.full(np.ones(3), A)
    Xh = T.full(np.ones(2), Ah)
    dense = np.sum((Xh - Xa) ** 2) / np.sum(Xa ** 2)
    assert abs(L.kruskal_loss(Ah, A) - dense) < 1e-12 * max(1.0, dense)
    assert abs(L.kruskal_loss(A, A)) < 1e-13


def test_kruskal_grad_matches_finite_differences():
    rng = np.random.default_rng(6)
    I = (4, 3, 5)
    A = random_factors(rng, I, 2)
    Ah = random_factors(rng, I, 2)
    _, g = L.kruskal_loss_grad(Ah, A)
    h = 1e-6
    for k in range(3):
        for i in range(I[k]):
            for r in range(2):
                P = [a.copy() for a in Ah]
                M = [a.copy() for a in Ah]
                P[k][i, r] += h
                M[k][i, r] -= h
                fd = (L.kruskal_loss(P, A) - L.kruskal_loss(M, A)) / (2 * h)
                assert abs(fd - g[k][i, r]) < 1e-7 * max(1.0, abs(fd)), (k, i, r)


def test_cosine_loss_equals_dense_cosine_and_grad_matches_fd():
    rng = np.random.default_rng(15)
    I = (4, 3, 5)
    A = random_factors(rng, I, 3)
    Ah = random_factors(rng, I, 2)
    Xa = T.full(np.ones(3), A).ravel()
    Xh = T.full(np.ones(2), Ah).ravel()
    dense = 1.0 - (Xa @ Xh) ** 2 / ((Xa @ Xa) * (Xh @ Xh))
    assert abs(L.kruskal_cosine_loss(Ah, A) - dense) < 1e-12
    # invariant to the scale of the prediction
    assert abs(L.kruskal_cosine_loss([3.0 * Ah[0], Ah[1], Ah[2]], A) - dense) < 1e-12
    loss, g = L.kruskal_cosine_loss_grad(Ah, A)
    assert abs(loss - dense) < 1e-12
    h = 1e-6
    for k in range(3):
        for i in range(I[k]):
            for r in range(2):
                P = [a.copy() for a in Ah]
                M = [a.copy() for a in Ah]
                P[k][i, r] += h
                M[k][i, r] -= h
                fd = (L.kruskal_cosine_loss(P, A) - L.kruskal_cosine_loss(M, A)) / (2 * h)
                assert abs(fd - g[k][i, r]) < 1e-7 * max(1.0, abs(fd)), (k, i, r)


def tiny_net(rng, din=6, h=5, dout=3 * 4 * 2):
    return (rng.standard_normal((h, din)) * 0.5, rng.standard_normal(h) * 0.1,
            rng.standard_normal((h, h)) * 0.5, rng.standard_normal(h) * 0.1,
            rng.standard_normal((dout, h)) * 0.5, rng.standard_normal(dout) * 0.1)


def net_loss(params, x, targets, I, R):
    y, _ = L.mlp_forward(params, x)
    loss, _ = L.batch_loss_grad(y, targets, I, R)
    return loss


def test_mlp_backward_matches_finite_differences():
    rng = np.random.default_rng(7)
    I, R = (4, 4, 4), 2
    params = list(tiny_net(rng))
    x = rng.standard_normal((3, 6))
    targets = [random_factors(rng, I, R) for _ in range(3)]
    y, cache = L.mlp_forward(params, x)
    _, dy = L.batch_loss_grad(y, targets, I, R)
    grads = L.mlp_backward(params, cache, dy)
    h = 1e-6
    for p, g in zip(params, grads):
        flat = p.reshape(-1)
        gf = g.reshape(-1)
        for idx in range(0, flat.size, max(1, flat.size // 7)):
            old = flat[idx]
            flat[idx] = old + h
            lp = net_loss(params, x, targets, I, R)
            flat[idx] = old - h
            lm = net_loss(params, x, targets, I, R)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - gf[idx]) < 1e-6 * max(1.0, abs(fd)), (p.shape, idx, fd, gf[idx])


def test_mlp_forward_is_the_composition():
    rng = np.random.default_rng(8)
    params = tiny_net(rng)
    x = rng.standard_normal((2, 6))
    y, _ = L.mlp_forward(params, x)
    W1, b1, W2, b2, W3, b3 = params
    for b in range(2):
        h1 = [max(0.0, sum(W1[o, i] * x[b, i] for i in range(6)) + b1[o]) for o in range(5)]
        h2 = [max(0.0, sum(W2[o, i] * h1[i] for i in range(5)) + b2[o]) for o in range(5)]
        for o in range(W3.shape[0]):
            ref = sum(W3[o, i] * h2[i] for i in range(5)) + b3[o]
            assert abs(y[b, o] - ref) < 1e-12


def test_adam_first_step_closed_form():
    """At t = 1 the bias-corrected moments are g and g^2, so the step is
    -lr * g / (|g| + eps)."""
    g = np.array([0.3, -2.0, 1e-3])
    w0 = np.array([1.0, 2.0, 3.0])
    w, m, v = L.adam_step(w0, g, np.zeros(3), np.zeros(3), 1, 0.01)
    np.testing.assert_allclose(w, w0 - 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


def test_planted_gradient_sign_is_caught():
    """A sign error in the cross term of the Kruskal gradient fails the
    finite-difference pin."""
    rng = np.random.default_rng(9)
    I = (3, 3, 3)
    A = random_factors(rng, I, 2)
    Ah = random_factors(rng, I, 2)
    aa = L.kruskal_inner(A, A)
    G = (Ah[1].T @ Ah[1]) * (Ah[2].T @ Ah[2])
    H = (Ah[1].T @ A[1]) * (Ah[2].T @ A[2])
    wrong = (2.0 * Ah[0] @ G + 2.0 * A[0] @ H.T) / aa
    h = 1e-6
    P = [a.copy() for a in Ah]
    M = [a.copy() for a in Ah]
    P[0][0, 0] += h
    M[0][0, 0] -= h
    fd = (L.kruskal_loss(P, A) - L.kruskal_loss(M, A)) / (2 * h)
    assert abs(fd - wrong[0, 0]) > 1e-4


def test_hosvd_start_spans_the_factor_subspace():
    """For an exact rank-R tensor the randomized HOSVD start spans the mode-k
    column space of the ground-truth factor, which is also the leading-R left
    singular subspace of X_(k) (projectors compared)."""
    import oracle.learned as OLm
    from oracle import tensor as T
    g = np.random.default_rng(4)
    shape, R = (12, 10, 9), 3
    A = [g.standard_normal((s, R)) for s in shape]
    X = T.full(np.ones(R), A)
    Om = [g.standard_normal((s, R)) for s in shape]
    Qs = OLm.hosvd_start(X, Om, R)
    for k in range(3):
        P = Qs[k] @ Qs[k].T
        Qa, _ = np.linalg.qr(A[k])
        np.testing.assert_allclose(P, Qa @ Qa.T, rtol=0, atol=1e-12)
        U, _, _ = np.linalg.svd(T.unfold(X, k), full_matrices=False)
        np.testing.assert_allclose(P, U[:, :R] @ U[:, :R].T, rtol=0, atol=1e-12)
        np.testing.assert_allclose(Qs[k].T @ Qs[k], np.eye(R), rtol=0, atol=1e-13)


def test_hosvd_start_is_the_qr_of_the_random_mttkrp():
    """W_k written out by index loops (sum over i_j, i_l of X times products
    of Omega entries), then its QR: equal to the oracle's start."""
    import itertools
    import oracle.learned as OLm
    g = np.random.default_rng(5)
    shape, R = (4, 3, 5), 2
    X = g.standard_normal(shape)
    Om = [g.standard_normal((s, R)) for s in shape]
    for k in range(3):
        W = np.zeros((shape[k], R))
        for idx in itertools.product(*[range(s) for s in shape]):
            for r in range(R):
                v = X[idx]
                for j in range(3):
                    if j != k:
                        v *= Om[j][idx[j], r]
                W[idx[k], r] += v
        Q, _ = np.linalg.qr(W)
        np.testing.assert_allclose(OLm.hosvd_start(X, Om, R, modes=[k])[k], Q, rtol=0, atol=1e-13)
