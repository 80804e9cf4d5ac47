"""The no-allocation Multi-TTM (cpqr_multittm_noalloc: static per-device
scratch instead of a workspace) against cpqr_multittm with a workspace, on
two calls in a row -- the second with a smaller input, so it runs over
scratch the first call left behind -- in FP32 and FP64, bit for bit (same
kernels, same plan, fixed-order sums).  Also: a request larger than the
static scratch is refused before anything runs."""

import ctypes

import numpy as np
import pytest
import torch

from paper_2112_10855_amd import cpqr as C
from paper_2112_10855_amd import synth
from helpers import to_dev


def test_noalloc_refuses_requests_beyond_the_scratch():
    """Host-side check, nothing is enqueued (runs without a GPU)."""
    L = C.lib()
    I = C._i64_array((1000, 1000, 1000))
    assert L.cpqr_multittm_work(3, I, 0, 16, C.PREC_F64) > C.NOALLOC_SCRATCH_BYTES
    P = ctypes.c_void_p(256)
    Qs = (ctypes.c_void_p * 3)(256, 256, 256)
    rc = L.cpqr_multittm_noalloc(3, I, C.F32, P, 0, 16, Qs, C.PREC_F64, P, None)
    assert rc == -4
    assert b"static array" in L.cpqr_last_error()


@pytest.mark.gpu
@pytest.mark.parametrize("prec", [C.PREC_F32, C.PREC_F64, C.PREC_BF16X2])
def test_noalloc_matches_workspace_entry_point(prec):
    cases = [((300, 260, 140), 16), ((64, 50, 30), 5)]  # second call smaller
    for call, (shape, R) in enumerate(cases):
        g = np.random.default_rng(100 + call)
        X = g.standard_normal(shape).astype(np.float32 if prec != C.PREC_F64 else np.float64)
        Qs = [synth.orthonormal_columns(s, R, 90 + 10 * call + k) for k, s in enumerate(shape)]
        Xd = to_dev(X, torch.float32 if X.dtype == np.float32 else torch.float64)
        Qd = [to_dev(q) for q in Qs]
        for n in range(3):
            Qn = [None if k == n else Qd[k] for k in range(3)]
            Yw = C.cpqr_multittm(Xd, Qn, n, prec)
            Yn = C.cpqr_multittm_noalloc(Xd, Qn, n, prec)
            torch.cuda.synchronize()
            assert Yw.shape == Yn.shape
            same = torch.equal(Yw.contiguous().view(torch.uint8), Yn.contiguous().view(torch.uint8))
            assert same, (call, shape, n, float((Yw - Yn).abs().max()))


@pytest.mark.gpu
def test_noalloc_into_caller_output_at_the_workload_size():
    """The 1000^3 FP32 rank-16 Multi-TTM fits the static scratch (about
    71 MB): Y passed in by the caller, so the call allocates nothing; the
    result equals the workspace entry point's."""
    n1, R = 1000, 16
    g = torch.Generator(device="cuda").manual_seed(5)
    Xd = torch.randn(n1 ** 3, device="cuda", generator=g, dtype=torch.float32).view(n1, n1, n1).permute(2, 1, 0)
    Qd = [C.colmajor(torch.randn(n1, R, device="cuda", generator=g, dtype=torch.float64)) for _ in range(3)]
    for n in range(3):
        Qn = [None if k == n else Qd[k] for k in range(3)]
        Y = C.empty_colmajor((n1, R * R), torch.float32, Xd.device)
        Yw = C.cpqr_multittm(Xd, Qn, n, C.PREC_F32)
        out = C.cpqr_multittm_noalloc(Xd, Qn, n, C.PREC_F32, Y=Y)
        torch.cuda.synchronize()
        assert out.data_ptr() == Y.data_ptr()
        assert torch.equal(Yw, Y)
