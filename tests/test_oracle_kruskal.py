"""Pins of the Kruskal-input oracle (section 3.3.2) and of the structured QR
of V_n (section 3.3.3, eq. kr-id).

Each Kruskal-input quantity is checked against the dense oracle on the
expanded tensor full(mu, V), itself pinned by index loops: W_n against
Y_(n) Q_0 from the dense Multi-TTM, the MTTKRP against the dense MTTKRP,
||X||^2 against the sum of squares, and whole CP-ALS-QR / CP-ALS runs against
the dense runs (equal up to rounding in exact arithmetic).  The structured
QR is checked against its defining properties: Q_0 R_0 = V_n with Q_0
orthonormal and R_0 upper triangular, and equality with the dense QR after
fixing column signs (a thin QR of a full-rank matrix is unique up to them).
Planted mistakes (Khatri-Rao operands swapped in the chain, a dropped weight)
must fail these pins."""

import numpy as np
import pytest

import oracle.cp_als as OA
import oracle.cp_als_qr as OQ
import oracle.kruskal as OK
from oracle import tensor as T
from paper_2112_10855_amd import synth


def rng(seed):
    return np.random.default_rng(seed)


def sign_fix(Qm, Rm):
    d = np.sign(np.diag(Rm))
    d[d == 0] = 1.0
    return Qm * d[None, :], Rm * d[:, None]


def random_kruskal(shape, S, seed, signed=True):
    g = rng(seed)
    V = [g.standard_normal((s, S)) for s in shape]
    mu = g.standard_normal(S) if signed else np.abs(g.standard_normal(S)) + 0.1
    return mu, V


def tri_factors(N, R, seed):
    g = rng(seed)
    return [OQ.factor_qr(g.standard_normal((R + 3, R)))[1] for _ in range(N)]


@pytest.mark.parametrize("N,R", [(2, 4), (3, 3), (3, 5), (4, 3), (4, 4), (5, 2), (5, 3), (6, 2)])
def test_structured_qr_of_khatri_rao(N, R):
    Rs = tri_factors(N, R, 10 * N + R)
    for n in range(N):
        Qs, R0 = OK.krp_qr_structured(Rs, n)
        assert len(Qs) == N - 2
        Q0 = OK.q0_from_structured(Qs, R)
        V = OQ.krp_of_r(Rs, n)
        assert Q0.shape == (R ** (N - 1), R)
        np.testing.assert_allclose(Q0 @ R0, V, rtol=0, atol=1e-13 * np.abs(V).max())
        np.testing.assert_allclose(Q0.T @ Q0, np.eye(R), rtol=0, atol=1e-14)
        assert np.all(np.tril(R0, -1) == 0)
        a, b = sign_fix(Q0, R0)
        ao, bo = sign_fix(*OQ.krp_qr(Rs, n))
        np.testing.assert_allclose(b, bo, rtol=0, atol=1e-12 * np.abs(bo).max())
        np.testing.assert_allclose(a, ao, rtol=0, atol=1e-11)


def test_structured_qr_keeps_the_sparsity_of_v():
    """Column r of V_n has (r+1)^{N-1} nonzeros (a Kronecker product of N-1
    columns of triangles, section 3.3.3); Q_0 from the structured factors has
    the same pattern (no fill-in): entry (i, r) of Q_0 is zero wherever
    column r of V_n is structurally zero."""
    N, R = 4, 4
    Rs = tri_factors(N, R, 99)
    V = OQ.krp_of_r(Rs, 0)
    Q0 = OK.q0_from_structured(OK.krp_qr_structured(Rs, 0)[0], R)
    for r in range(R):
        assert np.count_nonzero(V[:, r]) == (r + 1) ** (N - 1)
    pattern = np.abs(V) > 0
    assert np.all(np.abs(Q0[~pattern]) < 1e-14)


@pytest.mark.parametrize("shape,S,R", [((5, 4, 6), 7, 3), ((4, 3, 5, 4), 6, 3), ((3, 4, 3, 3, 4), 5, 2),
                                       ((6, 5), 4, 3)])
def test_w_kruskal_against_dense(shape, S, R):
    mu, V = random_kruskal(shape, S, sum(shape) + S)
    X = T.full(mu, V)
    N = len(shape)
    g = rng(7)
    Qf = [OQ.factor_qr(g.standard_normal((s, R)))[0] for s in shape]
    Rs = tri_factors(N, R, 8)
    for n in range(N):
        Qs, _ = OK.krp_qr_structured(Rs, n)
        Q0 = OK.q0_from_structured(Qs, R)
        ref = OQ.apply_q0(OQ.multittm_unfolded(X, [None if k == n else Qf[k] for k in range(N)], n), Q0)
        got = OK.w_kruskal(mu, V, Qf, Qs, n)
        np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12 * np.abs(ref).max())


@pytest.mark.parametrize("shape,S,R", [((5, 4, 6), 7, 3), ((4, 3, 5, 4), 6, 4), ((6, 5), 4, 3)])
def test_mttkrp_and_norm_kruskal_against_dense(shape, S, R):
    mu, V = random_kruskal(shape, S, 3 * S + R)
    X = T.full(mu, V)
    g = rng(5)
    A = [g.standard_normal((s, R)) for s in shape]
    for n in range(len(shape)):
        ref = T.mttkrp(X, A, n)
        np.testing.assert_allclose(OK.mttkrp_kruskal(mu, V, A, n), ref, rtol=0, atol=1e-12 * np.abs(ref).max())
    np.testing.assert_allclose(OK.norm2_kruskal(mu, V), float(np.sum(X * X)), rtol=1e-13)
    lam = g.standard_normal(R)
    np.testing.assert_allclose(OK.inner_kruskal(mu, V, lam, A), float(np.sum(X * T.full(lam, A))), rtol=1e-12)
    rel = OK.error_gram(mu, V, lam, A)
    np.testing.assert_allclose(rel, T.norm(X - T.full(lam, A)) / T.norm(X), rtol=1e-10)


@pytest.mark.parametrize("solver", ["qr", "svd"])
@pytest.mark.parametrize("N,n,R", [(3, 6, 3), (4, 5, 4), (5, 4, 5)])
def test_cp_als_qr_kruskal_matches_dense_on_sine_of_sums(solver, N, n, R):
    """The expanded sine-of-sums tensor (section 4.3): the Kruskal-input
    iteration reproduces the dense oracle's relative errors and model."""
    mu, V = synth.sine_of_sums_expanded(N, n)
    X = synth.sine_of_sums(N, n)
    init = [rng(40 + N).standard_normal((n, R)) for _ in range(N)]
    lk, Ak, hk = OK.cp_als_qr_kruskal(mu, V, init, maxiters=8, solver=solver, error="direct")
    ld, Ad, hd = OQ.cp_als_qr(X, init, maxiters=8, solver=solver, error="direct")
    np.testing.assert_allclose(hk, hd, rtol=0, atol=1e-12)
    Xk, Xd = T.full(lk, Ak), T.full(ld, Ad)
    assert T.norm(Xk - Xd) / T.norm(Xd) < 1e-11


@pytest.mark.parametrize("solver", ["chol", "pinv"])
def test_cp_als_kruskal_matches_dense(solver):
    mu, V = random_kruskal((6, 5, 7, 4), 9, 31, signed=True)
    X = T.full(mu, V)
    init = [rng(32).standard_normal((s, 3)) for s in (6, 5, 7, 4)]
    lk, Ak, hk = OK.cp_als_kruskal(mu, V, init, maxiters=6, solver=solver, error="efficient")
    ld, Ad, hd = OA.cp_als(X, init, maxiters=6, solver=solver, error="efficient")
    np.testing.assert_allclose(hk, hd, rtol=0, atol=1e-10)
    assert T.norm(T.full(lk, Ak) - T.full(ld, Ad)) / T.norm(T.full(ld, Ad)) < 1e-10


def test_error_forms_agree():
    mu, V = random_kruskal((5, 6, 4), 6, 77)
    init = [rng(78).standard_normal((s, 3)) for s in (5, 6, 4)]
    _, _, he = OK.cp_als_qr_kruskal(mu, V, init, maxiters=5, error="efficient")
    _, _, hg = OK.cp_als_qr_kruskal(mu, V, init, maxiters=5, error="gram")
    _, _, hd = OK.cp_als_qr_kruskal(mu, V, init, maxiters=5, error="direct")
    np.testing.assert_allclose(np.square(he), np.square(hd), rtol=0, atol=1e-12)
    np.testing.assert_allclose(np.square(hg), np.square(hd), rtol=0, atol=1e-12)


def test_planted_swapped_chain_operands_are_caught(monkeypatch):
    """C_j formed as C_{j-1} (.) B_{a_j} (the wrong index fastest) must fail
    the dense comparison."""
    mu, V = random_kruskal((4, 3, 5, 4), 6, 11)
    X = T.full(mu, V)
    g = rng(12)
    R = 3
    Qf = [OQ.factor_qr(g.standard_normal((s, R)))[0] for s in (4, 3, 5, 4)]
    Rs = tri_factors(4, R, 13)
    Qs, _ = OK.krp_qr_structured(Rs, 0)
    ref = OQ.apply_q0(OQ.multittm_unfolded(X, [None] + Qf[1:], 0), OK.q0_from_structured(Qs, R))
    real = T.khatri_rao
    monkeypatch.setattr(T, "khatri_rao", lambda A, B: real(B, A))
    bad = OK.w_kruskal(mu, V, Qf, Qs, 0)
    assert np.abs(bad - ref).max() > 1e-3 * np.abs(ref).max()


def test_planted_dropped_weights_are_caught():
    mu, V = random_kruskal((4, 5, 3), 5, 21)
    X = T.full(mu, V)
    A = [rng(22).standard_normal((s, 2)) for s in (4, 5, 3)]
    bad = OK.mttkrp_kruskal(np.ones_like(mu), V, A, 1)
    assert np.abs(bad - T.mttkrp(X, A, 1)).max() > 1e-3
