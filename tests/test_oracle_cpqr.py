"""Pins for the CP-ALS-QR oracle (Alg. 2) and its comparator (Alg. 1) against
what the paper and the mathematics fix: the structure of the QR of a
Khatri-Rao product (eq. Z_qr), the Gram identity, the least-squares
definition of every mode update (eq. ls_n) computed by an unrelated route,
the pseudo-inverse solution on rank-deficient problems, agreement with the
normal equations on well-conditioned problems, exact recovery, the two error
forms, ALS monotonicity and invariances.  The last group plants plausible
mistakes in the oracle and checks that a pin fails."""

import numpy as np
import pytest

import oracle.cp_als_qr as Q
import oracle.cp_als as ALS
from oracle import costs
from oracle import tensor as T
from paper_2112_10855_amd import synth


def rand_factors(shape, R, seed):
    rng = np.random.default_rng(seed)
    return [rng.standard_normal((s, R)) for s in shape]


# ---------------------------------------------------------------- pin checks
# Each returns an error figure; tests compare it with a tolerance and the
# planted-mistake tests check it goes above that tolerance.

def pin_krp_qr(shape, R, n, seed=0):
    """eq. (Z_qr): Z_n = (Q_N kron .. kron Q_1) Q_0 R_0 with orthonormal
    columns and upper-triangular R_0; R_0 equals the positive-diagonal
    triangular factor of Z_n obtained through Cholesky of Z_n^T Z_n."""
    N = len(shape)
    A = rand_factors(shape, R, seed)
    Qs, Rs = zip(*[Q.factor_qr(a) for a in A])
    Q0, R0 = Q.krp_qr(list(Rs), n)
    Z = T.khatri_rao_list([A[k] for k in reversed(range(N)) if k != n])
    Qbig = T.kron_list([Qs[k] for k in reversed(range(N)) if k != n]) @ Q0
    err = np.linalg.norm(Qbig @ R0 - Z) / np.linalg.norm(Z)
    err = max(err, np.linalg.norm(Qbig.T @ Qbig - np.eye(R)))
    err = max(err, np.abs(np.tril(R0, -1)).max())
    D = np.sign(np.diag(R0))
    Rc = np.linalg.cholesky(Z.T @ Z).T
    err = max(err, np.linalg.norm(D[:, None] * R0 - Rc) / np.linalg.norm(Rc))
    return err


def pin_mode_update_lstsq(shape, R, n, seed=0, solver="qr"):
    """eq. (ls_n): the mode update equals the least-squares solution computed
    by LAPACK's SVD-based lstsq on the explicit Khatri-Rao matrix Z_n."""
    N = len(shape)
    rng = np.random.default_rng(seed + 100)
    X = rng.standard_normal(shape)
    A = rand_factors(shape, R, seed)
    st = Q.init_state(A)
    for k in range(N):  # give mode n real neighbours: update modes before n
        if k == n:
            break
        Q.mode_update(X, st, k, solver=solver)
    Z = T.khatri_rao_list([st.A[k] for k in reversed(range(N)) if k != n])
    ref = np.linalg.lstsq(Z, T.unfold(X, n).T, rcond=None)[0].T
    out = Q.mode_update(X, st, n, solver=solver)
    err = np.linalg.norm(out["Ahat"] - ref) / np.linalg.norm(ref)
    # the normalized factor has unit 2-norm columns (eq. cp)
    err = max(err, np.abs(np.sqrt(np.sum(st.A[n] ** 2, axis=0)) - 1).max())
    err = max(err, np.linalg.norm(st.A[n] * st.lam[None, :] - ref) / np.linalg.norm(ref))
    return err


def lstsq_by_entries(X, A, n):
    """min over B of sum over all entries of (X[i] - sum_r B[i_n, r] prod_{k != n}
    A_k[i_k, r])^2, one small least-squares problem per i_n with one equation
    per tensor entry: no unfolding and no Khatri-Rao ordering involved."""
    import itertools
    N = X.ndim
    others = [k for k in range(N) if k != n]
    B = np.zeros((X.shape[n], A[0].shape[1]))
    for i_n in range(X.shape[n]):
        rows, rhs = [], []
        for rest in itertools.product(*[range(X.shape[k]) for k in others]):
            idx = [0] * N
            idx[n] = i_n
            z = np.ones(A[0].shape[1])
            for k, i_k in zip(others, rest):
                idx[k] = i_k
                z = z * A[k][i_k]
            rows.append(z)
            rhs.append(X[tuple(idx)])
        B[i_n] = np.linalg.lstsq(np.array(rows), np.array(rhs), rcond=None)[0]
    return B


def pin_als_update_lstsq(shape, R, n, seed=0, solver="chol"):
    """Alg. 1's mode update (normal equations by Cholesky, or the
    pseudo-inverse of S_n) equals the least-squares solution of eq. (ls_n)
    from LAPACK's SVD-based lstsq on the explicit Khatri-Rao matrix Z_n, and
    leaves unit columns, lambda and the Gram matrix of the new factor."""
    N = len(shape)
    rng = np.random.default_rng(seed + 200)
    X = rng.standard_normal(shape)
    A = rand_factors(shape, R, seed)
    G = [a.T @ a for a in A]
    for k in range(n):  # give mode n updated neighbours
        ALS.mode_update(X, A, G, k, solver=solver)
    ref = lstsq_by_entries(X, A, n)
    Ahat, lam, M, S = ALS.mode_update(X, A, G, n, solver=solver)
    err = np.linalg.norm(Ahat - ref) / np.linalg.norm(ref)
    err = max(err, np.linalg.norm(A[n] * lam[None, :] - ref) / np.linalg.norm(ref))
    err = max(err, np.abs(np.sqrt(np.sum(A[n] ** 2, axis=0)) - 1).max())
    err = max(err, np.abs(G[n] - A[n].T @ A[n]).max())
    return err


def pin_als_error_forms(seed=0, solver="chol"):
    """Alg. 1's efficient error (||X||^2 - 2 <M_N, Ahat_N> + <S_N, diag(lam)
    G_N diag(lam)>) against the residual of the dense model, on squares."""
    d = synth.workload_small(noise=1e-2, seed_item=seed)
    X = d["X"]
    worst = 0.0
    for its in (1, 2, 4):
        lam, A, h = ALS.cp_als(X, d["init"], maxiters=its, solver=solver)
        dire = T.norm(X - T.full(lam, A)) / T.norm(X)
        worst = max(worst, abs(h[-1] ** 2 - dire ** 2))
    return worst


def pin_error_forms(seed=0):
    """section 3.3.1: the efficient and the direct relative error agree;
    compared on squared errors, where the identity holds exactly."""
    d = synth.workload_small(noise=1e-2, seed_item=seed)
    X = d["X"]
    st = Q.init_state(d["init"])
    worst = 0.0
    for _ in range(3):
        eff, _ = Q.sweep(X, st, error="efficient")
        dire = Q.error_direct(X, st.lam, st.A)
        worst = max(worst, abs(eff ** 2 - dire ** 2))
    return worst


# ------------------------------------------------------------------- the pins

@pytest.mark.parametrize("shape,R", [((5, 6, 4), 3), ((4, 3, 5, 3), 2), ((3, 4, 2, 3), 4), ((3, 3, 3, 3, 3), 2),
                                     ((7, 8, 9), 5)])
def test_krp_qr_structure(shape, R):
    for n in range(len(shape)):
        assert pin_krp_qr(shape, R, n) < 1e-12


@pytest.mark.parametrize("shape,R", [((6, 5, 7), 3), ((4, 5, 3, 4), 3), ((3, 4, 3, 2, 3), 2), ((9, 8, 7), 5)])
@pytest.mark.parametrize("solver", ["qr", "svd"])
def test_mode_update_is_least_squares(shape, R, solver):
    for n in range(len(shape)):
        assert pin_mode_update_lstsq(shape, R, n, solver=solver) < 1e-11


def test_gram_identity():
    """R_0^T R_0 = Hadamard product of A_k^T A_k over k != n (section 2.3 gives
    Z_n^T Z_n as that Hadamard product, and Z_n^T Z_n = R_0^T R_0)."""
    shape, R = (6, 5, 4, 3), 3
    A = rand_factors(shape, R, 3)
    Rs = [Q.factor_qr(a)[1] for a in A]
    for n in range(4):
        _, R0 = Q.krp_qr(Rs, n)
        H = T.hadamard_list([A[k].T @ A[k] for k in range(4) if k != n])
        np.testing.assert_allclose(R0.T @ R0, H, rtol=1e-12, atol=1e-12 * np.abs(H).max())


def test_w_times_r0_is_mttkrp():
    """W_n R_0 = X_(n) Z_n (section 3.3.1): applying Q_0 after the Multi-TTM
    and multiplying by R_0 gives the MTTKRP."""
    shape, R = (5, 4, 6), 3
    rng = np.random.default_rng(9)
    X = rng.standard_normal(shape)
    A = rand_factors(shape, R, 4)
    Qs, Rs = zip(*[Q.factor_qr(a) for a in A])
    for n in range(3):
        Q0, R0 = Q.krp_qr(list(Rs), n)
        W = Q.apply_q0(Q.multittm_unfolded(X, list(Qs), n), Q0)
        M = T.mttkrp(X, A, n)
        np.testing.assert_allclose(W @ R0, M, rtol=0, atol=1e-12 * np.abs(M).max())


def test_multittm_unfolded_kron_form():
    """Y_(n) = X_(n) (Q_N kron ... kron Q_1) skipping n (eq. multittm with
    U_k = Q_k^T)."""
    shape, R = (4, 5, 3, 2), 2
    rng = np.random.default_rng(10)
    X = rng.standard_normal(shape)
    Qs = [Q.factor_qr(a)[0] for a in rand_factors(shape, R, 5)]
    for n in range(4):
        K = T.kron_list([Qs[k] for k in reversed(range(4)) if k != n])
        np.testing.assert_allclose(Q.multittm_unfolded(X, Qs, n), T.unfold(X, n) @ K, rtol=0, atol=1e-12)


def test_svd_variant_is_pinv_on_rank_deficient():
    """CP-ALS-QR-SVD gives the minimum-norm solution X_(n) pinv(Z_n^T) when
    Z_n is rank deficient (section 2.1, section 3.1); duplicated columns in
    every factor make Z_n rank deficient and R_0 singular."""
    shape, R = (6, 5, 7), 4
    rng = np.random.default_rng(11)
    A = rand_factors(shape, R, 6)
    for a in A:
        a[:, 1] = a[:, 0]
    X = rng.standard_normal(shape)
    st = Q.init_state(A)
    n = 0
    Z = T.khatri_rao_list([A[k] for k in reversed(range(3)) if k != n])
    assert np.linalg.matrix_rank(Z) == R - 1
    ref = T.unfold(X, n) @ np.linalg.pinv(Z.T)
    out = Q.mode_update(X, st.copy(), n, solver="svd")
    assert out["kept"] == R - 1
    assert out["status"] & Q.RANK_TRUNCATED
    np.testing.assert_allclose(out["Ahat"], ref, rtol=0, atol=1e-9 * np.abs(ref).max())


@pytest.mark.parametrize("shape,R", [((6, 5, 7), 3), ((4, 5, 3, 4), 3), ((3, 4, 3, 2, 3), 2), ((9, 8, 7), 5)])
@pytest.mark.parametrize("solver", ["chol", "pinv"])
def test_als_mode_update_is_least_squares(shape, R, solver):
    for n in range(len(shape)):
        assert pin_als_update_lstsq(shape, R, n, solver=solver) < 1e-10


@pytest.mark.parametrize("solver", ["chol", "pinv"])
def test_als_error_forms_agree(solver):
    assert pin_als_error_forms(solver=solver) < 1e-13


def test_als_pinv_is_min_norm_on_rank_deficient():
    """CP-ALS-PINV: with Z_n rank deficient (a duplicated column in every
    factor), M_n pinv(S_n) = X_(n) Z_n pinv(Z_n^T Z_n) = X_(n) pinv(Z_n^T),
    the minimum-norm least-squares solution (section 2.3)."""
    shape, R = (6, 5, 7), 4
    rng = np.random.default_rng(12)
    A = rand_factors(shape, R, 7)
    for a in A:
        a[:, 2] = a[:, 1]
    X = rng.standard_normal(shape)
    G = [a.T @ a for a in A]
    n = 1
    Z = T.khatri_rao_list([A[k] for k in reversed(range(3)) if k != n])
    assert np.linalg.matrix_rank(Z) == R - 1
    ref = T.unfold(X, n) @ np.linalg.pinv(Z.T)
    Ahat, lam, M, S = ALS.mode_update(X, A, G, n, solver="pinv")
    np.testing.assert_allclose(Ahat, ref, rtol=0, atol=1e-9 * np.abs(ref).max())


def test_planted_gram_of_mode_n_in_hadamard_is_caught(monkeypatch):
    """Taking every Gram matrix into S_n (mode n's own included) is caught."""
    real = T.hadamard_list
    monkeypatch.setattr(T, "hadamard_list", lambda mats: real(list(mats) + [np.eye(mats[0].shape[0]) * 1.5]))
    assert pin_als_update_lstsq((6, 5, 7), 3, 1) > 1e-3


def test_planted_mttkrp_order_is_caught(monkeypatch):
    """A Khatri-Rao product taken from mode 1 up instead of mode N down."""
    real = T.khatri_rao_list
    monkeypatch.setattr(T, "khatri_rao_list", lambda mats: real(list(reversed(mats))))
    monkeypatch.setattr(ALS, "T", T)
    assert pin_als_update_lstsq((6, 5, 7), 3, 0) > 1e-3 or pin_als_update_lstsq((6, 5, 7), 3, 2) > 1e-3


def test_qr_matches_normal_equations_trajectory():
    """CP-ALS-QR and CP-ALS compute the same iterates in exact arithmetic;
    on a well-conditioned problem (50^3, rank 5, noise 1e-4) their relative
    error histories and final models agree closely (section 1, section 4.2)."""
    d = synth.workload_small()
    X = d["X"]
    lq, Aq, hq = Q.cp_als_qr(X, d["init"], maxiters=25)
    la, Aa, ha = ALS.cp_als(X, d["init"], maxiters=25)
    np.testing.assert_allclose(hq, ha, rtol=0, atol=1e-8)
    Mq, Ma = T.full(lq, Aq), T.full(la, Aa)
    assert T.norm(Mq - Ma) / T.norm(Ma) < 1e-8
    assert hq[-1] < 2e-4  # at the noise level


def test_exact_low_rank_recovery():
    """A noise-free rank-5 tensor is recovered to relative error <= 1e-10
    (direct error, section 3.3.1)."""
    d = synth.workload_small(noise=0.0)
    lam, A, hist = Q.cp_als_qr(d["X"], d["init"], maxiters=300, tol=1e-16, error="direct")
    assert Q.error_direct(d["X"], lam, A) <= 1e-10


def test_error_forms_agree():
    assert pin_error_forms() < 1e-13


def test_monotone_residual():
    """Each mode update minimizes the residual over one block exactly
    (eq. ls_n), so ||X - Xhat|| never increases from one update to the next."""
    d = synth.workload_small(noise=1e-2)
    X = d["X"]
    st = Q.init_state(d["init"])
    Q.mode_update(X, st, 0)  # after this every factor is defined
    prev = T.norm(X - T.full(st.lam, st.A))
    for _ in range(4):
        for n in (1, 2, 0):
            Q.mode_update(X, st, n)
            r = T.norm(X - T.full(st.lam, st.A))
            assert r <= prev * (1 + 1e-12)
            prev = r


def test_invariance_to_init_scaling_and_qr_signs(monkeypatch):
    """Scaling the initial columns and flipping QR signs leaves the normalized
    iterates unchanged (the LS solution is unique; signs of Q_k, Q_0 cancel)."""
    d = synth.workload_small(noise=1e-3)
    X = d["X"]
    lam0, A0, h0 = Q.cp_als_qr(X, d["init"], maxiters=5)
    scaled = [a * np.linspace(0.5, 3.0, a.shape[1])[None, :] for a in d["init"]]
    lam1, A1, h1 = Q.cp_als_qr(X, scaled, maxiters=5)
    np.testing.assert_allclose(lam1, lam0, rtol=1e-10)
    for a, b in zip(A0, A1):
        np.testing.assert_allclose(a, b, rtol=0, atol=1e-10)

    orig_fqr, orig_kqr = Q.factor_qr, Q.krp_qr

    def flipped(fn):
        def g(*args):
            Qm, Rm = fn(*args)
            s = np.where(np.arange(Rm.shape[0]) % 2 == 0, -1.0, 1.0)
            return Qm * s[None, :], s[:, None] * Rm
        return g

    monkeypatch.setattr(Q, "factor_qr", flipped(orig_fqr))
    monkeypatch.setattr(Q, "krp_qr", flipped(orig_kqr))
    lam2, A2, h2 = Q.cp_als_qr(X, d["init"], maxiters=5)
    np.testing.assert_allclose(lam2, lam0, rtol=1e-10)
    for a, b in zip(A0, A2):
        np.testing.assert_allclose(a, b, rtol=0, atol=1e-10)
    np.testing.assert_allclose(h2, h0, rtol=0, atol=1e-12)


def test_ttm_cost_model():
    """The simulated TTM sequence cost equals eq. (TTMcost) for the
    decreasing-size order."""
    for shape in [(700, 700, 700), (300, 300, 300, 300), (75,) * 5, (50, 60, 40), (200, 100, 300, 50)]:
        for n in range(len(shape)):
            for R in (1, 5, 16, 32):
                a = costs.ttm_sequence_flops(shape, n, R)
                b = costs.ttm_cost_closed_form(shape, n, R)
                assert abs(a - b) <= 1e-9 * b


def counted_householder_qr(M):
    """Textbook Householder QR of an m x n matrix with Q formed explicitly by
    backward accumulation, run on the actual numbers and counting every
    floating-point addition, multiplication, division and square root it
    performs.  Returns (Q, R, flop count).  Independent of the cost formula:
    the count is what the loops execute."""
    A = np.array(M, dtype=np.float64)
    m, n = A.shape
    flops = 0
    vs, taus = [], []
    for j in range(n):
        x = A[j:, j].copy()
        nrm = np.sqrt(np.dot(x, x))
        flops += 2 * len(x)                       # squares, sum, sqrt
        alpha = -nrm if x[0] >= 0 else nrm
        v = x.copy()
        v[0] -= alpha
        flops += 1
        vv = np.dot(v, v)
        flops += 2 * len(v)
        tau = 0.0 if vv == 0 else 2.0 / vv
        flops += 1
        for c in range(j + 1, n):                # A(j:, c) -= tau v (v^T A(j:, c))
            d = np.dot(v, A[j:, c])
            A[j:, c] -= tau * d * v
            flops += 2 * len(v) + 1 + 2 * len(v)
        A[j, j] = alpha                          # H_j x = alpha e_1
        A[j + 1:, j] = 0.0
        vs.append(v)
        taus.append(tau)
    Qm = np.eye(m, n)
    for j in reversed(range(n)):                 # Q = H_0 .. H_{n-1} [I; 0]
        v, tau = vs[j], taus[j]
        for c in range(j, n):
            d = np.dot(v, Qm[j:, c])
            Qm[j:, c] -= tau * d * v
            flops += 2 * len(v) + 1 + 2 * len(v)
    return Qm, np.triu(A[:n, :]), flops


@pytest.mark.parametrize("N,R", [(3, 4), (3, 6), (4, 3), (4, 5), (5, 3), (6, 2)])
def test_krp_qr_cost_against_counted_householder(N, R):
    """eq. (QRcost): the QR of the R^{N-1} x R matrix V_n with Q_0 formed
    costs 4 R^{N+1} flops to leading order.  A Householder QR that counts the
    operations it performs on V_n agrees with that figure up to the terms of
    order R^3 (the triangle: 4 R^3 / 3) and R^N (the reflector norms: about
    4 m R), and the counted QR really factors V_n.  The bound is tight enough
    that 2 R^{N+1} or 4 R^N would fail it."""
    rng = np.random.default_rng(N * 10 + R)
    Rs = [Q.factor_qr(rng.standard_normal((R + 2, R)))[1] for _ in range(N)]
    V = Q.krp_of_r(Rs, 0)
    m = R ** (N - 1)
    assert V.shape == (m, R)
    Qm, Rm, flops = counted_householder_qr(V)
    assert np.linalg.norm(Qm @ Rm - V) <= 1e-13 * np.linalg.norm(V)
    lead = costs.krp_qr_flops(N, R)
    lower = 4.0 * m * R + 4.0 * R ** 3 / 3.0 + 8.0 * R * R
    assert abs(flops - lead) <= lower, (flops, lead, lower)


def test_krp_qr_cost_leading_term_dominates():
    """The terms below eq. (QRcost)'s leading one are of relative size 1/R
    (reflector norms) and R^{2-N} (the triangle): with N = 3 and growing R
    the counted flops approach 4 R^{N+1} from above."""
    ratios = []
    for R in (4, 8, 16):
        rng = np.random.default_rng(R)
        Rs = [Q.factor_qr(rng.standard_normal((R + 2, R)))[1] for _ in range(3)]
        flops = counted_householder_qr(Q.krp_of_r(Rs, 0))[2]
        ratios.append(flops / costs.krp_qr_flops(3, R))
    assert ratios[0] > ratios[1] > ratios[2] > 1.0
    assert ratios[2] - 1.0 < 0.1, ratios


# ---------------------------------------------------------- planted mistakes

def test_planted_wrong_krp_order_is_caught(monkeypatch):
    def bad(Rs, n):
        return T.khatri_rao_list([Rs[k] for k in range(len(Rs)) if k != n])
    monkeypatch.setattr(Q, "krp_of_r", bad)
    assert pin_mode_update_lstsq((6, 5, 7), 3, 1) > 1e-6


def test_planted_wrong_solve_orientation_is_caught(monkeypatch):
    import scipy.linalg

    def bad(W, R0):
        return scipy.linalg.solve_triangular(R0, W.T, lower=False, trans="T").T, 0
    monkeypatch.setattr(Q, "solve_qr", bad)
    assert pin_mode_update_lstsq((6, 5, 7), 3, 0) > 1e-6


def test_planted_missing_transpose_in_multittm_is_caught(monkeypatch):
    def bad(X, Qs, n, order=None):
        U = [None if q is None else q[:, ::-1].T for q in Qs]  # permuted columns
        return T.unfold(T.multittm(X, U, n, order=order), n)
    monkeypatch.setattr(Q, "multittm_unfolded", bad)
    assert pin_mode_update_lstsq((6, 5, 7), 3, 2) > 1e-6


def test_planted_error_term_is_caught(monkeypatch):
    def bad(xnorm2, W, Ahat, R0, lam, RN):
        ip = float(np.sum(W * (Ahat @ R0.T)))
        nn = float(np.sum((R0.T @ R0) * (RN.T @ RN)))  # lambda scaling dropped
        return float(np.sqrt(max(xnorm2 - 2 * ip + nn, 0)) / np.sqrt(xnorm2))
    monkeypatch.setattr(Q, "error_efficient", bad)
    assert pin_error_forms() > 1e-6


def test_planted_wrong_norm_is_caught(monkeypatch):
    def bad(Ahat):
        lam = np.sum(np.abs(Ahat), axis=0)
        return Ahat / lam[None, :], lam
    monkeypatch.setattr(Q, "normalize", bad)
    assert pin_mode_update_lstsq((6, 5, 7), 3, 0) > 1e-6


def test_planted_krp_qr_without_q0_is_caught(monkeypatch):
    orig = Q.krp_qr

    def bad(Rs, n):
        Q0, R0 = orig(Rs, n)
        return Q0, np.triu(Q.krp_of_r(Rs, n)[: R0.shape[0]])
    monkeypatch.setattr(Q, "krp_qr", bad)
    assert pin_krp_qr((5, 6, 4), 3, 0) > 1e-6
