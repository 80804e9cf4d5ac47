"""GPU path on Kruskal-form inputs (section 3.3.2) against the FP64 oracle.

* cpqr_kruskal_w, cpqr_kruskal_mttkrp, cpqr_kruskal_norm2 and
  cpqr_kruskal_full entry by entry against oracle.kruskal (itself pinned to
  the dense oracle), with tolerances relative to the sum of the magnitudes of
  the products that make up each entry (the same computation on |mu|, |V|,
  |Q|): every rounding error is a multiple of those products.
* Whole CP-ALS-QR / CP-ALS-QR-SVD and CP-ALS / CP-ALS-PINV runs on Kruskal
  inputs against the oracle's Kruskal-input runs: squared relative errors
  (efficient form) to 1e-10 and dense models to 1e-9.
* The 10-way sine of sums at n = 8 (section 4.3.3): the rank-512 input,
  rank 10, a few sweeps of each algorithm against the oracle, and sampled
  entries of the dense 8^10 tensor formed on the device."""

import numpy as np
import pytest
import torch

import oracle.kruskal as OK
import oracle.cp_als_qr as OQ
from oracle import tensor as OT
from paper_2112_10855_amd import cpqr as C
from paper_2112_10855_amd import synth
from helpers import assert_entrywise, relnorm, to_dev, to_np

pytestmark = pytest.mark.gpu


def rng(seed):
    return np.random.default_rng(seed)


def random_kruskal(shape, S, seed):
    g = rng(seed)
    return g.standard_normal(S), [g.standard_normal((s, S)) for s in shape]


def dev_kruskal(mu, V):
    return to_dev(mu), [to_dev(v) for v in V]


@pytest.mark.parametrize("shape,S,R", [((9, 8, 7), 5, 3), ((6, 7, 5, 6), 11, 4), ((5, 4, 6, 5, 4), 7, 3),
                                       ((4, 3, 4, 3, 4, 3), 9, 3), ((40, 35, 30), 64, 12), ((3,) * 10, 20, 2)])
def test_kruskal_w(shape, S, R):
    mu, V = random_kruskal(shape, S, sum(shape) + S)
    N = len(shape)
    g = rng(5)
    Qf = [OQ.factor_qr(g.standard_normal((s, R)))[0] for s in shape]
    Rs = [OQ.factor_qr(g.standard_normal((R + 2, R)))[1] for _ in shape]
    mud, Vd = dev_kruskal(mu, V)
    for n in sorted({0, N // 2, N - 1}):
        Qc, _ = C.cpqr_krp_qr_chain([to_dev(r) for r in Rs], n)
        Qs = list(to_np(Qc))
        W = to_np(C.cpqr_kruskal_w(mud, Vd, [None if k == n else to_dev(Qf[k]) for k in range(N)], Qc, n))
        ref = OK.w_kruskal(mu, V, Qf, Qs, n)
        bound = OK.w_kruskal(np.abs(mu), [np.abs(v) for v in V], [np.abs(q) for q in Qf], [np.abs(q) for q in Qs], n)
        assert_entrywise(W, ref, bound, 1e-13, (shape, n))


@pytest.mark.parametrize("shape,S,R", [((9, 8, 7), 5, 3), ((6, 7, 5, 6), 11, 4), ((30, 20, 25), 40, 16),
                                       ((3,) * 10, 20, 2), ((50, 60), 9, 5)])
def test_kruskal_mttkrp_and_norm(shape, S, R):
    mu, V = random_kruskal(shape, S, 3 * S + R)
    N = len(shape)
    A = [rng(9 + k).standard_normal((s, R)) for k, s in enumerate(shape)]
    mud, Vd = dev_kruskal(mu, V)
    Ad = [to_dev(a) for a in A]
    for n in range(N):
        M = to_np(C.cpqr_kruskal_mttkrp(mud, Vd, [None if k == n else Ad[k] for k in range(N)], n))
        ref = OK.mttkrp_kruskal(mu, V, A, n)
        bound = OK.mttkrp_kruskal(np.abs(mu), [np.abs(v) for v in V], [np.abs(a) for a in A], n)
        assert_entrywise(M, ref, bound, 1e-13, (shape, n))
    x2 = float(to_np(C.cpqr_kruskal_norm2(mud, Vd))[0])
    bound = OK.norm2_kruskal(np.abs(mu), [np.abs(v) for v in V])
    assert abs(x2 - OK.norm2_kruskal(mu, V)) <= 1e-13 * bound


@pytest.mark.parametrize("shape,S", [((7, 5, 6), 4), ((65, 70, 3), 9), ((5, 4, 3, 6), 33), ((3,) * 8, 12),
                                     ((130, 129), 17)])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_kruskal_full(shape, S, dtype):
    mu, V = random_kruskal(shape, S, S + len(shape))
    X = to_np(C.cpqr_kruskal_full(*dev_kruskal(mu, V), dtype=dtype)).astype(np.float64)
    ref = OT.full(mu, V)
    bound = OT.full(np.abs(mu), [np.abs(v) for v in V])
    tol = 1e-14 if dtype == torch.float64 else 2.0 ** -24 + 1e-14
    assert_entrywise(X, ref, bound, tol, shape)


@pytest.mark.parametrize("I,R", [(8, 10), (3, 7), (1, 4), (20, 32), (31, 32)])
def test_factor_qr_of_wide_factor(I, R):
    """I < R: the QR of A padded with zero rows.  Q's columns I.. and Rk's rows
    I.. are exactly zero; the rest equals LAPACK's QR of A (I x I orthonormal
    Q, I x R trapezoidal R) up to the signs of the rows of R."""
    A = rng(I * 100 + R).standard_normal((I, R))
    Qd, Rd = C.cpqr_factor_qr(to_dev(A))
    Q, Rk = to_np(Qd), to_np(Rd)
    Qo, Ro = OQ.factor_qr(A)
    assert np.all(Q[:, I:] == 0.0) and np.all(Rk[I:, :] == 0.0)
    assert np.all(np.tril(Rk, -1) == 0.0)
    d = np.sign(np.diag(Rk[:I, :I]))
    do = np.sign(np.diag(Ro[:, :I]))
    np.testing.assert_allclose(Q[:, :I] * d[None, :], Qo * do[None, :], rtol=0, atol=1e-13)
    np.testing.assert_allclose(Rk[:I, :] * d[:, None], Ro * do[:, None], rtol=0, atol=1e-13 * np.abs(Ro).max())
    np.testing.assert_allclose(Q @ Rk, A, rtol=0, atol=1e-13 * np.abs(A).max())


def gpu_run(algo, mu, V, init, sweeps, error_mode=C.ERROR_EFFICIENT, X=None):
    kr = dev_kruskal(mu, V)
    if algo in ("qr", "svd"):
        st, hist = C.cp_als_qr(X, init, maxiters=sweeps, prec=C.PREC_F64, use_svd=algo == "svd",
                               error_mode=error_mode, kruskal=kr)
    else:
        st, hist = C.cp_als(X, init, maxiters=sweeps, prec=C.PREC_F64, solver=algo, error_mode=error_mode,
                            kruskal=kr)
    torch.cuda.synchronize()
    return to_np(st.lam), [to_np(a) for a in st.A], np.array(hist), int(st.status.item())


def oracle_run(algo, mu, V, init, sweeps, error):
    if algo in ("qr", "svd"):
        return OK.cp_als_qr_kruskal(mu, V, init, maxiters=sweeps, solver=algo, error=error)
    return OK.cp_als_kruskal(mu, V, init, maxiters=sweeps, solver=algo, error=error)


@pytest.mark.parametrize("algo", ["qr", "svd", "chol", "pinv"])
@pytest.mark.parametrize("shape,S,R", [((12, 10, 9), 6, 4), ((8, 7, 6, 9), 10, 5), ((6, 5, 6, 5, 6), 8, 3),
                                       ((20, 17), 7, 5), ((4, 6, 3, 5), 9, 7)])
def test_kruskal_sweeps_against_oracle(algo, shape, S, R):
    mu, V = random_kruskal(shape, S, 71 + S)
    init = [rng(72).standard_normal((s, R)) for s in shape]
    lam, A, hist, status = gpu_run(algo, mu, V, init, 8)
    lo, Ao, ho = oracle_run(algo, mu, V, init, 8, "efficient")
    np.testing.assert_allclose(np.square(hist), np.square(ho), rtol=0, atol=1e-10)
    # dense models: the Gram-matrix form of the distance resolves only ~1e-8
    assert relnorm(OT.full(lam, A), OT.full(lo, Ao)) < 1e-9


@pytest.mark.parametrize("algo", ["qr", "chol"])
def test_kruskal_direct_error_with_dense_tensor(algo):
    """The direct error reads the dense tensor (formed on the device from the
    factors); it matches the oracle's direct error on the same iterates."""
    shape, S, R = (10, 9, 8, 7), 12, 4
    mu, V = random_kruskal(shape, S, 404)
    init = [rng(405).standard_normal((s, R)) for s in shape]
    Xd = C.cpqr_kruskal_full(*dev_kruskal(mu, V))
    lam, A, hist, _ = gpu_run(algo, mu, V, init, 6, error_mode=C.ERROR_DIRECT, X=Xd)
    lo, Ao, ho = oracle_run(algo, mu, V, init, 6, "direct")
    np.testing.assert_allclose(hist, ho, rtol=1e-9, atol=1e-14)


def test_kruskal_sine_of_sums_matches_dense_path():
    """The expanded 4-way sine of sums (section 4.3): the Kruskal-input sweeps
    and the dense-input sweeps from the same start give the same errors."""
    N, n, R = 4, 16, 4
    mu, V = synth.sine_of_sums_expanded(N, n)
    X = synth.sine_of_sums(N, n)
    init = [rng(300).standard_normal((n, R)) for _ in range(N)]
    for algo in ("qr", "svd", "chol", "pinv"):
        _, _, hk, _ = gpu_run(algo, mu, V, init, 12, error_mode=C.ERROR_DIRECT, X=to_dev(X))
        if algo in ("qr", "svd"):
            st, hd = C.cp_als_qr(to_dev(X), init, maxiters=12, prec=C.PREC_F64, use_svd=algo == "svd",
                                 error_mode=C.ERROR_DIRECT)
        else:
            st, hd = C.cp_als(to_dev(X), init, maxiters=12, prec=C.PREC_F64, solver=algo, error_mode=C.ERROR_DIRECT)
        np.testing.assert_allclose(hk, hd, rtol=1e-8, atol=1e-13)


@pytest.fixture(scope="module")
def sinsum10():
    N, n = 10, 8
    mu, V = synth.sine_of_sums_expanded(N, n)
    return N, n, mu, V


@pytest.mark.parametrize("algo", ["qr", "svd", "chol", "pinv"])
def test_sine_of_sums_10way_against_oracle(sinsum10, algo):
    """Section 4.3.3: N = 10, n = 8, the rank-512 input, rank 10; three sweeps
    from a seeded start against the oracle's Kruskal-input run (squared
    relative errors to 1e-10, models to 1e-8)."""
    N, n, mu, V = sinsum10
    R = N
    init = [rng(1000).standard_normal((n, R)) for _ in range(N)]
    lam, A, hist, _ = gpu_run(algo, mu, V, init, 3)
    lo, Ao, ho = oracle_run(algo, mu, V, init, 3, "gram")
    print("[sinsum10] %s gpu %s oracle %s" % (algo, hist, ho), flush=True)
    np.testing.assert_allclose(np.square(hist), np.square(ho), rtol=0, atol=1e-10)
    # unit-norm columns with the signs the solve gives: compared directly (the
    # Gram-matrix form of the model distance resolves only ~1e-8)
    assert relnorm(lam, lo) < 1e-8
    for k in range(N):
        assert relnorm(A[k], Ao[k]) < 1e-8, k


def test_sine_of_sums_10way_dense_tensor_sampled(sinsum10):
    """The dense 8^10 FP64 tensor (8.6 GB) formed on the device: sampled
    entries against the sine of the sum of the grid points (the closed form
    the rank-512 expansion represents) and against the Kruskal sum."""
    N, n, mu, V = sinsum10
    Xd = C.cpqr_kruskal_full(*dev_kruskal(mu, V))
    torch.cuda.synchronize()
    g = rng(17)
    idx = g.integers(0, n, size=(2000, N))
    flat = np.zeros(len(idx), dtype=np.int64)
    for k in range(N - 1, -1, -1):
        flat = flat * n + idx[:, k]
    got = to_np(Xd.permute(*reversed(range(N))).reshape(-1)[torch.from_numpy(flat).cuda()])
    x = synth.sine_of_sums_grid(n)
    closed = np.sin(x[idx].sum(axis=1))
    kr = np.array([np.sum(mu * np.prod([V[k][i[k]] for k in range(N)], axis=0)) for i in idx])
    bound = np.array([np.sum(np.abs(mu) * np.prod([np.abs(V[k][i[k]]) for k in range(N)], axis=0)) for i in idx])
    assert np.all(np.abs(got - kr) <= 1e-14 * bound)
    assert np.abs(got - closed).max() < 1e-12
    del Xd
    torch.cuda.empty_cache()
