"""GPU Multi-TTM in the reduced-precision forms (split bfloat16 hi/lo with
three products, and plain bfloat16), FP32 accumulation, against the FP64
oracle.  The GPU's relative error must be within a factor 3 of the error of
the oracle's emulation of the same form (same operand rounding, exact sums,
FP32 intermediates); accumulation order differs, so bitwise equality is not
expected.  Every entry of the GPU result (and of the emulation) is also
checked against the exact Multi-TTM within the per-contraction error bound of
its form, relative to the magnitude bound |X| x |Q| of that entry.  The FP32
form is checked against the 1e-5 contract for reference.
"""

import numpy as np
import pytest
import torch

import oracle.cp_als_qr as OQ
from oracle import precision as OP
from paper_2112_10855_amd import cpqr as C
from paper_2112_10855_amd import synth
from helpers import abs_bound_multittm, assert_entrywise, multittm_tol_lowp, relnorm, to_dev, to_np

pytestmark = pytest.mark.gpu

# the last two: the mode-3 update's first contraction is over the middle
# mode of short slabs (whole-slab workgroups)
SHAPES = [((64, 64, 64), 16), ((100, 37, 52), 5), ((40, 36, 33, 20), 12), ((130, 20, 24), 32), ((33, 47, 29), 8),
          ((16, 200, 8), 16), ((100, 80, 260), 12), ((60, 50, 300), 5)]


@pytest.mark.parametrize("shape,R", SHAPES)
@pytest.mark.parametrize("mode", ["bf16x2", "bf16"])
def test_multittm_lowp_error_matches_emulation(shape, R, mode):
    g = np.random.default_rng(sum(shape) + R)
    X = g.standard_normal(shape).astype(np.float32)
    Rr = min(R, min(shape))
    Qs = [synth.orthonormal_columns(s, Rr, 40 + k) for k, s in enumerate(shape)]
    Xd = to_dev(X, torch.float32)
    prec = C.PREC_BF16X2 if mode == "bf16x2" else C.PREC_BF16
    for n in range(len(shape)):
        Y = to_np(C.cpqr_multittm(Xd, [None if k == n else to_dev(Qs[k]) for k in range(len(shape))], n, prec))
        exact = OQ.multittm_unfolded(X.astype(np.float64), Qs, n)
        emul = OP.multittm_lowp(X, Qs, n, mode)
        e_gpu, e_emul = relnorm(Y, exact), relnorm(emul, exact)
        assert e_emul / 3 <= e_gpu <= 3 * e_emul, (n, e_gpu, e_emul)
        bound = abs_bound_multittm(X, Qs, n)
        tol = multittm_tol_lowp(shape, n, mode)
        assert_entrywise(emul, exact, bound, tol, ("emulation", shape, n))
        assert_entrywise(Y, exact, bound, tol, ("gpu", shape, n))


def test_precision_ordering_on_one_tensor():
    """FP32 < split bfloat16 < plain bfloat16 in error.  Measured on this
    tensor: 2.3e-7, 6.3e-6 and 3.3e-3; the bounds are those values with a
    factor 2-4 of margin.  FP32 and split bfloat16 meet the 1e-5 contract;
    plain bfloat16 misses its 1e-3 contract on the raw Multi-TTM (about 2^-9
    per product, summed over 16 x 16 terms), which is asserted as a miss so
    that a change in it is noticed."""
    g = np.random.default_rng(11)
    shape = (96, 80, 72)
    X = g.standard_normal(shape).astype(np.float32)
    Qs = [synth.orthonormal_columns(s, 16, 60 + k) for k, s in enumerate(shape)]
    Xd = to_dev(X, torch.float32)
    errs = {}
    for name, prec in [("f32", C.PREC_F32), ("bf16x2", C.PREC_BF16X2), ("bf16", C.PREC_BF16)]:
        Y = to_np(C.cpqr_multittm(Xd, [None, to_dev(Qs[1]), to_dev(Qs[2])], 0, prec))
        errs[name] = relnorm(Y, OQ.multittm_unfolded(X.astype(np.float64), Qs, 0))
    print("[precision] Multi-TTM errors:", {k: "%.2e" % v for k, v in errs.items()})
    assert errs["f32"] < 1e-6
    assert errs["bf16x2"] < 2e-5
    assert 1e-3 < errs["bf16"] < 6.6e-3
    assert errs["f32"] < errs["bf16x2"] < errs["bf16"]


@pytest.mark.parametrize("prec,tol,tol_err", [(C.PREC_BF16X2, 1e-5, 1e-5), (C.PREC_BF16, 1e-3, 5e-4)])
def test_sweeps_in_reduced_precision(prec, tol, tol_err):
    """CP-ALS-QR with the reduced-precision Multi-TTM still fits the small
    noisy workload: the final model is within tol of the FP64 oracle's.
    Measured (deterministic: fixed seeds, fixed-order reductions): split
    bfloat16 1.9e-6 on the model and 2e-9 on the error; plain bfloat16 9.0e-4
    on the model -- inside the 1e-3 plain-bfloat16 contract, which applies to
    the fitted model -- and 3.5e-4 on the error (its raw Multi-TTM error,
    3-5e-3, misses 1e-3).  The bounds are the contract (model) and the
    measured value with margin (error)."""
    d = synth.workload_small(noise=1e-3)
    X = d["X"].astype(np.float32)
    st, hist = C.cp_als_qr(to_dev(X, torch.float32), d["init"], maxiters=15, prec=prec,
                           error_mode=C.ERROR_DIRECT)
    lo, Ao, ho = OQ.cp_als_qr(X.astype(np.float64), d["init"], maxiters=15, error="direct")
    from oracle import tensor as OT
    lam = to_np(st.lam)
    A = [to_np(a) for a in st.A]
    dist = relnorm(OT.full(lam, A), OT.full(lo, Ao))
    print("[precision] prec %d: model distance %.2e, final relerr %.6e vs %.6e" % (prec, dist, hist[-1], ho[-1]))
    assert dist < tol
    assert abs(hist[-1] - ho[-1]) < tol_err
