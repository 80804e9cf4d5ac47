"""The sine-of-sums workload of section 4.3 on the GPU: the four ALS
algorithms (CP-ALS, CP-ALS-PINV, CP-ALS-QR, CP-ALS-QR-SVD) fit the rank-N
representation of sin(x_1 + ... + x_N) from one shared random start, FP64,
with the relative error taken directly.

Parity: at N = 4, n = 16 the GPU error histories and models match the
oracle's.  Perturbing X by 2e-16 (relative, random) moves the oracle's own
histories by at most 1.1e-13 on this problem, so the FP64 bar of the other
sweep tests (1e-10) applies.  Claim (the paper's figures for N = 4 and 5):
the QR-based algorithms end lower than the normal-equations ones.  The rank-N
form is not unique and how ill-conditioned the representation the iteration
approaches is depends on the start (from some starts every algorithm reaches
1e-15), so the claim is checked on the N = 5, n = 32 grid from the start the
benchmark uses, where the gap is about two orders of magnitude; reductions
are fixed-order, so the run is reproducible."""

import numpy as np
import pytest
import torch

import oracle.cp_als as OA
import oracle.cp_als_qr as OQ
from oracle import tensor as OT
from paper_2112_10855_amd import cpqr as C
from paper_2112_10855_amd import synth
from helpers import relnorm, to_dev, to_np

pytestmark = pytest.mark.gpu

ALGS = ["als", "pinv", "qr", "qrsvd"]


def run_gpu(alg, Xd, init, iters):
    kw = dict(maxiters=iters, prec=C.PREC_F64, error_mode=C.ERROR_DIRECT)
    if alg in ("als", "pinv"):
        st, hist = C.cp_als(Xd, init, solver="chol" if alg == "als" else "pinv", **kw)
    else:
        st, hist = C.cp_als_qr(Xd, init, use_svd=alg == "qrsvd", **kw)
    torch.cuda.synchronize()
    return to_np(st.lam), [to_np(a) for a in st.A], np.array(hist)


def run_oracle(alg, X, init, iters):
    if alg in ("als", "pinv"):
        return OA.cp_als(X, init, maxiters=iters, solver="chol" if alg == "als" else "pinv", error="direct")
    return OQ.cp_als_qr(X, init, maxiters=iters, solver="svd" if alg == "qrsvd" else "qr", error="direct")


@pytest.mark.parametrize("alg", ALGS)
def test_parity_4way_n16(alg):
    N, n = 4, 16
    X = synth.sine_of_sums(N, n)
    init = synth.init_factors((n,) * N, N, 4300)
    lam, A, hist = run_gpu(alg, to_dev(X, torch.float64), init, 15)
    lo, Ao, ho = run_oracle(alg, X, init, 15)
    np.testing.assert_allclose(hist, ho, rtol=0, atol=1e-10)
    assert relnorm(OT.full(lam, A), OT.full(lo, Ao)) < 1e-9
    assert hist[-1] < 1e-8  # converging to the exact rank-4 form


def test_qr_reaches_lower_error_5way_n32():
    N, n = 5, 32
    Xd = to_dev(synth.sine_of_sums(N, n), torch.float64)
    init = synth.init_factors((n,) * N, N, 4400 + 10 * N + n)
    final = {alg: run_gpu(alg, Xd, init, 40)[2][-1] for alg in ALGS}
    print({k: "%.2e" % v for k, v in final.items()})
    assert max(final["qr"], final["qrsvd"]) < 1e-13
    assert 10 * max(final["qr"], final["qrsvd"]) < min(final["als"], final["pinv"])


def test_hybrid_switches_to_qr_and_reaches_its_accuracy():
    """The hybrid solver on the same problem: CP-ALS until a Cholesky step
    proves cond(S_n) > 1e4, then CP-ALS-QR from the current factors.  The same
    inverse-iteration bound evaluated on the oracle's CP-ALS iterates first
    exceeds 1e4 in sweep 6 (1.7e4, with cond(S_n) = 6.3e4); after the switch
    the error reaches the QR level that CP-ALS alone does not."""
    N, n = 5, 32
    Xd = to_dev(synth.sine_of_sums(N, n), torch.float64)
    init = synth.init_factors((n,) * N, N, 4400 + 10 * N + n)
    st, hist, n_ne = C.cp_als_hybrid(Xd, init, maxiters=40, prec=C.PREC_F64, error_mode=C.ERROR_DIRECT)
    print("hybrid: %d normal-equations sweeps, final %.2e" % (n_ne, hist[-1]))
    assert n_ne == 6
    assert len(hist) == 40
    assert hist[-1] < 1e-13
