"""GPU parity of each C-ABI entry point against the FP64 oracle, on seeded
inputs that span several tiles, ragged tails and the degenerate cases.

Tolerances:
  * FP64 paths: 1e-12 relative (Householder QR and FP64 sums of at most a
    few thousand terms; the oracle uses LAPACK, so results agree to a small
    multiple of K * 2^-53).
  * FP32 Multi-TTM: the tensor is stored in FP32 (the oracle reads the same
    bytes in FP64); Q is rounded to FP32 (relative 2^-24) and sums run in
    FP32 over at most K terms per contraction.  Multi-TTM and apply-Q_0
    results are checked entry by entry: |Y - Y_oracle| <= tol * (|X| x |Q|),
    the magnitude bound of that entry's products, with tol = 1e-5 (the FP32
    contract) or 1e-12 (FP64).
"""

import numpy as np
import pytest
import torch

import oracle.cp_als_qr as OQ
from oracle import tensor as OT
from paper_2112_10855_amd import cpqr as C
from paper_2112_10855_amd import synth
from helpers import abs_bound_multittm, assert_entrywise, multittm_tol_f32, relnorm, sign_fix, to_dev, to_np

pytestmark = pytest.mark.gpu


def rng(seed):
    return np.random.default_rng(seed)


# ------------------------------------------------------------------ factor QR

@pytest.mark.parametrize("I,R", [(50, 5), (64, 16), (65, 16), (1000, 16), (200, 32), (256, 10), (130, 3),
                                 (5000, 7), (100, 1), (2000, 32), (32, 32), (4097, 12), (129, 16), (257, 16),
                                 (2048, 16), (6000, 8), (1024, 8), (64, 32), (65, 32), (20000, 16),
                                 (100000, 3), (256, 16), (1024, 16), (1025, 16), (257, 32), (70000, 16),
                                 (70000, 32), (33000, 32),
                                 # ranks that fill the second half of the split WY factor only in part
                                 (64, 9), (150, 17), (300, 20), (1000, 24), (500, 31), (3000, 20)])
def test_factor_qr(I, R):
    A = rng(I * 100 + R).standard_normal((I, R))
    Q, Rk = C.cpqr_factor_qr(to_dev(A))
    Q, Rk = to_np(Q), to_np(Rk)
    assert np.abs(np.tril(Rk, -1)).max() == 0.0
    assert np.linalg.norm(Q.T @ Q - np.eye(R)) < 1e-13 * max(1, np.sqrt(R))
    assert relnorm(Q @ Rk, A) < 1e-14
    Qo, Ro = OQ.factor_qr(A)
    Qs, Rs = sign_fix(Q, Rk)
    Qos, Ros = sign_fix(Qo, Ro)
    assert relnorm(Rs, Ros) < 1e-12
    assert relnorm(Qs, Qos) < 1e-11


def test_factor_qr_rank_deficient():
    """Duplicated and zero columns: Q must still have orthonormal columns and
    Q R must reproduce A."""
    A = rng(7).standard_normal((300, 8))
    A[:, 3] = A[:, 1]
    A[:, 5] = 0.0
    Q, Rk = C.cpqr_factor_qr(to_dev(A))
    Q, Rk = to_np(Q), to_np(Rk)
    assert np.linalg.norm(Q.T @ Q - np.eye(8)) < 1e-13
    assert relnorm(Q @ Rk, A) < 1e-14


# ------------------------------------------------------------------ KRP QR

@pytest.mark.parametrize("N,R", [(3, 5), (3, 16), (4, 7), (2, 8), (5, 3), (3, 1), (4, 32), (3, 32), (6, 4),
                                 (5, 12)])
def test_krp_qr(N, R):
    g = rng(N * 1000 + R)
    Rs = [OQ.factor_qr(g.standard_normal((R + 3, R)))[1] for _ in range(N)]
    for n in sorted({0, N - 1, N // 2}):
        Q0, R0 = C.cpqr_krp_qr([to_dev(r) for r in Rs], n)
        Q0, R0 = to_np(Q0), to_np(R0)
        Q0o, R0o = OQ.krp_qr(Rs, n)
        assert np.abs(np.tril(R0, -1)).max() == 0.0
        assert np.linalg.norm(Q0.T @ Q0 - np.eye(R)) < 1e-12
        a, b = sign_fix(Q0, R0)
        ao, bo = sign_fix(Q0o, R0o)
        assert relnorm(b, bo) < 1e-11
        assert relnorm(a, ao) < 1e-10


# ------------------------------------------------------------------ Multi-TTM

SHAPES = [(33, 47, 29), (64, 64, 64), (100, 37, 52), (12, 9, 17, 8), (5, 6, 4, 7, 3), (130, 20, 24),
          (16, 200, 8), (7, 5)]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("R", [5, 16, 32])
def test_multittm_f32(shape, R):
    g = rng(hash((shape, R)) % (2 ** 31))
    X = g.standard_normal(shape).astype(np.float32)
    Rr = min(R, min(shape))
    Qs = [synth.orthonormal_columns(s, Rr, 10 * k + 1) for k, s in enumerate(shape)]
    Xd = to_dev(X, torch.float32)
    for n in range(len(shape)):
        Y = to_np(C.cpqr_multittm(Xd, [None if k == n else to_dev(Qs[k]) for k in range(len(shape))], n, C.PREC_F32))
        Yo = OQ.multittm_unfolded(X.astype(np.float64), Qs, n)
        assert Y.shape == Yo.shape
        assert_entrywise(Y, Yo, abs_bound_multittm(X, Qs, n), multittm_tol_f32(shape, n), (shape, R, n))


@pytest.mark.parametrize("shape", SHAPES[:6] + [(130, 20, 24), (16, 200, 8), (96, 64, 300)])
@pytest.mark.parametrize("xdtype", [np.float64, np.float32])
@pytest.mark.parametrize("Rw", [6, 16, 32])
def test_multittm_f64(shape, xdtype, Rw):
    """FP64 Multi-TTM: FP64 tensors stream through the FP64 matrix-core row
    tiles (one or two 16-column blocks, 64- or 128-row tiles, split K, with
    and without non-temporal loads), FP32 tensors through the vector-ALU
    kernel."""
    R = min(Rw, min(shape))
    g = rng(17)
    X = g.standard_normal(shape).astype(xdtype)
    Qs = [synth.orthonormal_columns(s, R, 10 * k + 2) for k, s in enumerate(shape)]
    Xd = to_dev(X, torch.float64 if xdtype == np.float64 else torch.float32)
    for n in range(len(shape)):
        Y = to_np(C.cpqr_multittm(Xd, [None if k == n else to_dev(Qs[k]) for k in range(len(shape))], n, C.PREC_F64))
        Yo = OQ.multittm_unfolded(X.astype(np.float64), Qs, n)
        assert_entrywise(Y, Yo, abs_bound_multittm(X, Qs, n), 1e-12, (shape, n))


@pytest.mark.parametrize("shape,R", [((75, 33, 41), 16), ((35, 75, 29, 17), 12), ((17, 19, 23), 5), ((75, 75, 75), 32),
                                     ((45, 25, 35, 21, 19), 4), ((1001, 37, 19), 16), ((21, 300, 37), 24)])
def test_multittm_f64_rows_not_multiple_of_four(shape, R):
    """FP64 Multi-TTM whose contractions have P % 4 != 0 (odd mode sizes):
    rows loaded one by one by the row-tiled matrix-core kernel (P >= 16) or
    the vector-ALU kernel (smaller P), entry by entry against the oracle."""
    R = min(R, min(shape))
    g = rng(sum(shape) + R)
    X = g.standard_normal(shape)
    Qs = [synth.orthonormal_columns(s, R, 3 * k + 1) for k, s in enumerate(shape)]
    Xd = to_dev(X)
    for n in range(len(shape)):
        Y = to_np(C.cpqr_multittm(Xd, [None if k == n else to_dev(Qs[k]) for k in range(len(shape))], n, C.PREC_F64))
        Yo = OQ.multittm_unfolded(X, Qs, n)
        assert_entrywise(Y, Yo, abs_bound_multittm(X, Qs, n), 1e-12, (shape, n))


@pytest.mark.parametrize("shape,R", [((600, 301, 257), 16), ((600, 304, 257), 16), ((60, 50, 300), 5),
                                     ((100, 80, 260), 12), ((120, 100, 300), 32), ((1000, 600, 256), 24),
                                     ((200, 180, 256), 17), ((40, 36, 20, 16), 9), ((48, 40, 300), 32)])
def test_multittm_short_slabs(shape, R):
    """Every mode update of tensors whose first contraction is over mode 2
    with short slabs (P = I_1 <= 1024 rows, a multiple of 4, at least 256
    slabs).  For the updates of modes 3, 4, .. the first two contractions run
    fused, one workgroup per slab (64- and 128-row tiles, one or two
    16-column blocks, K tails, line-aligned and unaligned stretches, and a
    4-way tensor whose third contraction follows the fused pair)."""
    g = rng(sum(shape) + R)
    X = g.standard_normal(shape).astype(np.float32)
    Qs = [synth.orthonormal_columns(s, R, 10 * k + 3) for k, s in enumerate(shape)]
    Xd = to_dev(X, torch.float32)
    for n in range(len(shape)):
        Y = to_np(C.cpqr_multittm(Xd, [None if k == n else to_dev(Qs[k]) for k in range(len(shape))], n,
                                  C.PREC_F32))
        Yo = OQ.multittm_unfolded(X.astype(np.float64), Qs, n)
        assert_entrywise(Y, Yo, abs_bound_multittm(X, Qs, n), multittm_tol_f32(shape, n), (shape, n))


def test_multittm_general_matrices_elementwise():
    """Non-orthonormal operands and an element-by-element check against the
    brute-force sum on a tiny tensor."""
    g = rng(5)
    shape = (6, 8, 4)
    X = g.standard_normal(shape).astype(np.float32)
    Us = [g.standard_normal((s, 3)) for s in shape]
    Y = to_np(C.cpqr_multittm(to_dev(X, torch.float32), [to_dev(u) for u in Us], 1, C.PREC_F32))
    for i in range(8):
        for a in range(3):
            for c in range(3):
                v = sum(float(X[p, i, q]) * Us[0][p, a] * Us[2][q, c] for p in range(6) for q in range(4))
                assert abs(Y[i, a + 3 * c] - v) <= 1e-5 * (1 + abs(v))


# ------------------------------------------------------------------ apply Q0

@pytest.mark.parametrize("In,K,R", [(50, 25, 5), (1000, 256, 16), (200, 32768, 32), (37, 64, 8), (300, 1000, 10),
                                    (1000, 4096, 16), (50, 1331, 11), (130, 1025, 7)])
@pytest.mark.parametrize("ydt", [np.float32, np.float64])
def test_apply_q0(In, K, R, ydt):
    g = rng(In + K + R)
    Y = g.standard_normal((In, K)).astype(ydt)
    Q0 = synth.orthonormal_columns(K, R, 3)
    W = to_np(C.cpqr_apply_q0(to_dev(Y, torch.float32 if ydt == np.float32 else torch.float64), to_dev(Q0)))
    Wo = OQ.apply_q0(Y.astype(np.float64), Q0)
    assert_entrywise(W, Wo, np.abs(Y.astype(np.float64)) @ np.abs(Q0), 1e-12, (In, K, R))


# ------------------------------------------------------------------ solve

@pytest.mark.parametrize("In,R", [(50, 5), (1000, 16), (200, 32), (300, 1), (77, 13)])
@pytest.mark.parametrize("use_svd", [False, True])
def test_solve_rsvd(In, R, use_svd):
    g = rng(In * 7 + R)
    W = g.standard_normal((In, R))
    R0 = OQ.factor_qr(g.standard_normal((R + 5, R)))[1]
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    A, lam = C.cpqr_solve_rsvd(to_dev(W), to_dev(R0), use_svd=use_svd, status=status)
    if use_svd:
        Ah, kept, st = OQ.solve_svd(W, R0)
    else:
        Ah, st = OQ.solve_qr(W, R0)
    Ao, lamo = OQ.normalize(Ah)
    assert relnorm(to_np(lam), lamo) < 1e-11
    assert relnorm(to_np(A), Ao) < 1e-11
    assert int(status.item()) == 0


def test_solve_svd_rank_deficient_and_status():
    """Exactly singular R_0: the SVD solve drops the null direction like the
    oracle's pseudo-inverse; substitution flags the singular diagonal."""
    g = rng(9)
    R = 6
    B = g.standard_normal((20, R))
    B[:, 4] = B[:, 1]
    R0 = OQ.factor_qr(B)[1]
    R0[4, 4] = 0.0
    W = g.standard_normal((90, R))
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    A, lam = C.cpqr_solve_rsvd(to_dev(W), to_dev(R0), use_svd=True, status=status)
    Ah, kept, _ = OQ.solve_svd(W, R0)
    assert kept == R - 1
    Ao, lamo = OQ.normalize(Ah)
    assert relnorm(to_np(A) * to_np(lam)[None, :], Ah) < 1e-9
    assert int(status.item()) & C.STATUS_TRUNCATED
    status.zero_()
    C.cpqr_solve_rsvd(to_dev(W), to_dev(R0), use_svd=False, status=status)
    assert int(status.item()) & C.STATUS_SINGULAR


def test_zero_column_status():
    W = rng(3).standard_normal((40, 4))
    W[:, 2] = 0.0
    R0 = np.eye(4)
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    A, lam = C.cpqr_solve_rsvd(to_dev(W), to_dev(R0), status=status)
    assert to_np(lam)[2] == 0.0 and np.all(to_np(A)[:, 2] == 0.0)
    assert int(status.item()) & C.STATUS_ZERO_COLUMN


# ------------------------------------------------------------------ direct fit

@pytest.mark.parametrize("shape,R", [((50, 50, 50), 5), ((300, 7, 70), 16), ((9, 8, 7, 6), 3), ((1030, 3, 65), 32)])
@pytest.mark.parametrize("xdt", [np.float32, np.float64])
def test_fit_direct(shape, R, xdt):
    g = rng(sum(shape) + R)
    A = [g.standard_normal((s, R)) / np.sqrt(s) for s in shape]
    lam = g.random(R) + 0.5
    X = (OT.full(lam, A) + 0.01 * g.standard_normal(shape)).astype(xdt)
    out = to_np(C.cpqr_fit_direct(to_dev(X, torch.float32 if xdt == np.float32 else torch.float64), to_dev(lam),
                                  [to_dev(a) for a in A]))
    Xd = X.astype(np.float64)
    r2 = OT.norm(Xd - OT.full(lam, A)) ** 2
    x2 = OT.norm(Xd) ** 2
    assert abs(out[1] - x2) <= 1e-12 * x2
    assert abs(out[0] - r2) <= 1e-10 * r2


# ------------------------------------------------------------------ structured KRP QR

def chain_q0(Qc, N):
    """Q_0 = (I kron Q_2)(I kron Q_3) .. Q_{N-1} formed explicitly (test side)."""
    R = Qc.shape[2]
    Q0 = Qc[N - 3]
    for j in range(N - 4, -1, -1):  # Q_0 = (I_{R^{N-3-j}} kron Q_{j+2}) .. ; build from the right
        Q0 = np.kron(np.eye(R ** (N - 3 - j)), Qc[j]) @ Q0
    return Q0


@pytest.mark.parametrize("N,R", [(3, 5), (3, 16), (4, 7), (4, 32), (5, 3), (5, 12), (6, 4), (7, 3), (10, 2)])
def test_krp_qr_chain(N, R):
    """The structured QR (eq. kr-id applied step by step) against the oracle's
    dense QR of the explicit V_n: R_0 and Q_0 equal after fixing the signs of
    the columns, Q_0 orthonormal, Q_0 R_0 = V_n."""
    g = rng(N * 100 + R)
    Rs = [OQ.factor_qr(g.standard_normal((R + 3, R)))[1] for _ in range(N)]
    for n in sorted({0, N - 1, N // 2}):
        Qc, R0 = C.cpqr_krp_qr_chain([to_dev(r) for r in Rs], n)
        Qc, R0 = to_np(Qc), to_np(R0)
        assert Qc.shape == (N - 2, R * R, R)
        Q0 = chain_q0(Qc, N)
        Q0o, R0o = OQ.krp_qr(Rs, n)
        V = OQ.krp_of_r(Rs, n)
        assert np.abs(np.tril(R0, -1)).max() == 0.0
        assert np.linalg.norm(Q0.T @ Q0 - np.eye(R)) < 1e-12
        assert relnorm(Q0 @ R0, V) < 1e-13
        a, b = sign_fix(Q0, R0)
        ao, bo = sign_fix(Q0o, R0o)
        assert relnorm(b, bo) < 1e-11, relnorm(b, bo)
        assert relnorm(a, ao) < 1e-10, relnorm(a, ao)


@pytest.mark.parametrize("N,R", [(3, 6), (4, 32), (5, 3), (5, 12), (6, 4), (7, 3), (10, 2)])
def test_expand_q0(N, R):
    """Q_0 formed on the device from the structured factors equals the
    Kronecker product chain formed on the host, entry by entry."""
    g = rng(N * 31 + R)
    Rs = [OQ.factor_qr(g.standard_normal((R + 2, R)))[1] for _ in range(N)]
    Qc, R0 = C.cpqr_krp_qr_chain([to_dev(r) for r in Rs], N - 1)
    Q0 = to_np(C.cpqr_expand_q0(Qc, N))
    Qc_np = to_np(Qc)
    ref = chain_q0(Qc_np, N)
    Qa = np.abs(Qc_np)
    bound = Qa[N - 3]
    for j in range(N - 4, -1, -1):
        bound = np.kron(np.eye(R ** (N - 3 - j)), Qa[j]) @ bound
    assert_entrywise(Q0, ref, bound, 1e-13, (N, R))


@pytest.mark.parametrize("In,N,R", [(50, 4, 5), (200, 4, 32), (37, 5, 6), (130, 3, 16), (64, 6, 3)])
@pytest.mark.parametrize("ydt", [np.float32, np.float64])
def test_apply_q0_chain(In, N, R, ydt):
    """W = Y_(n) Q_0 through the structured factors equals the product with
    the explicit Q_0, entry by entry (FP64, magnitude bound |Y| |Q_0|)."""
    g = rng(In + N + R)
    Rs = [OQ.factor_qr(g.standard_normal((R + 3, R)))[1] for _ in range(N)]
    Qc, R0 = C.cpqr_krp_qr_chain([to_dev(r) for r in Rs], 0)
    Qc_np = to_np(Qc)
    Q0 = chain_q0(Qc_np, N)
    Y = g.standard_normal((In, R ** (N - 1))).astype(ydt)
    W = to_np(C.cpqr_apply_q0_chain(to_dev(Y, torch.float32 if ydt == np.float32 else torch.float64), Qc, N))
    Y64 = Y.astype(np.float64)
    assert_entrywise(W, Y64 @ Q0, np.abs(Y64) @ np.abs(Q0), 1e-12, (In, N, R))
