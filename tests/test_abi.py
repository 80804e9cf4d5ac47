"""The C-ABI library loads on a host without a GPU, exports every symbol
include/cpqr.h declares, and rejects bad arguments with the documented error
codes before touching the device (no compute calls here)."""

import ctypes
import os
import re

import pytest

from paper_2112_10855_amd import cpqr as C

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(C.LIBPATH):
        from paper_2112_10855_amd import build
        build.build()
    return C.lib()


def header_symbols():
    txt = open(os.path.join(ROOT, "include", "cpqr.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(cpqr_[a-z0-9_]+)\s*\(", txt)))


def test_every_declared_symbol_is_exported(L):
    syms = header_symbols()
    assert len(syms) >= 20
    for s in syms:
        assert hasattr(L, s), s
    assert set(syms) == set(C.EXPORTED)


def test_version(L):
    assert L.cpqr_version() == 100


def code(rc):
    return rc


def test_validation_codes(L):
    P = 4096  # fake, never dereferenced: validation fails first
    assert L.cpqr_factor_qr(10, 0, P, 10, P, 10, P, 10, P, 1 << 20, None) == -2
    assert L.cpqr_factor_qr(10, 33, P, 10, P, 10, P, 10, P, 1 << 20, None) == -2
    assert L.cpqr_factor_qr(0, 4, P, 10, P, 10, P, 10, P, 1 << 20, None) == -2
    assert L.cpqr_factor_qr(10, 4, None, 10, P, 10, P, 10, P, 1 << 20, None) == -1
    assert L.cpqr_factor_qr(10, 4, P, 9, P, 10, P, 10, P, 1 << 20, None) == -2
    # 5000 rows take a two-level tree, which needs a work buffer
    assert L.cpqr_factor_qr_work(1000, 4) == 0
    assert L.cpqr_factor_qr_work(5000, 4) > 16
    assert L.cpqr_factor_qr(5000, 4, P, 5000, P, 5000, P, 10, None, 0, None) == -4
    assert L.cpqr_factor_qr(5000, 4, P, 5000, P, 5000, P, 10, P + 8, 1 << 20, None) == -4
    assert L.cpqr_factor_qr(5000, 4, P, 5000, P, 5000, P, 10, P, 16, None) == -4
    assert b"too small" in L.cpqr_last_error()

    I = C._i64_array([10, 11, 12])
    Qs = C._ptr_array([None, None, None])
    assert L.cpqr_multittm(3, I, 0, P, 0, 4, Qs, 1, P, P, 1 << 30, None) == -1  # Q[1] NULL
    Qs = (ctypes.c_void_p * 3)(P, P, P)
    assert L.cpqr_multittm(3, I, 1, P, 0, 4, Qs, 1, P, P, 1 << 30, None) == -3  # F64 X with F32 prec
    assert L.cpqr_multittm(3, I, 0, P, 3, 4, Qs, 1, P, P, 1 << 30, None) == -1  # n out of range
    assert L.cpqr_multittm(1, I, 0, P, 0, 4, Qs, 1, P, P, 1 << 30, None) == -2  # N < 2
    assert L.cpqr_multittm(3, I, 0, P, 0, 4, Qs, 9, P, P, 1 << 30, None) == -1  # bad precision
    I0 = C._i64_array([10, 0, 12])
    assert L.cpqr_multittm(3, I0, 0, P, 0, 4, Qs, 1, P, P, 1 << 30, None) == -2

    assert L.cpqr_krp_qr(3, 3, 4, Qs, 4, P, P, P, 1 << 30, None) == -1
    assert L.cpqr_krp_qr(11, 0, 4, Qs, 4, P, P, P, 1 << 30, None) == -2
    assert L.cpqr_krp_qr(3, 0, 4, Qs, 3, P, P, P, 1 << 30, None) == -2
    assert L.cpqr_apply_q0(10, 3, 4, 0, P, P, P, P, 1 << 30, None) == -2
    assert L.cpqr_apply_q0(10, 16, 4, 7, P, P, P, P, 1 << 30, None) == -3
    assert L.cpqr_solve_rsvd(0, 4, P, P, 0, -1.0, P, P, None, P, 1 << 30, None) == -2
    assert L.cpqr_solve_rsvd(10, 4, None, P, 0, -1.0, P, P, None, P, 1 << 30, None) == -1
    assert L.cpqr_solve_rsvd(10, 4, P, P, 0, float("nan"), P, P, None, P, 1 << 30, None) == -1
    assert L.cpqr_fit_direct(3, I, 2, P, 4, P, Qs, P, P, 1 << 30, None) == -3

    p = C.Problem()
    p.N, p.R = 3, 4
    for k in range(3):
        p.I[k] = 10
        p.A[k] = p.Q[k] = p.Rf[k] = P
    p.X, p.lam, p.xdtype, p.prec, p.error_mode = P, P, 0, 1, 0
    assert L.cpqr_als_work(ctypes.byref(p)) > 0
    p.I[2] = 3  # smaller than the rank
    assert L.cpqr_als_work(ctypes.byref(p)) == 0
    assert L.cpqr_als_init(ctypes.byref(p), P, 1 << 30, None) == -2
    p.I[2] = 10
    p.error_mode = 5
    assert L.cpqr_als_sweep(ctypes.byref(p), 1, None, P, 1 << 30, None) == -1
    p.error_mode = 0
    assert L.cpqr_als_sweep(ctypes.byref(p), -1, None, P, 1 << 30, None) == -1
    assert L.cpqr_als_sweep(ctypes.byref(p), 1, None, P, 16, None) == -4
    assert L.cpqr_als_sweep(None, 1, None, P, 16, None) == -1


def test_validation_normal_equations(L):
    """Alg. 1 entry points: Q and Rf may be NULL (CP-ALS-QR still needs
    them); the rest of the problem is validated as for the QR sweep."""
    P = 4096
    p = C.Problem()
    p.N, p.R = 3, 4
    for k in range(3):
        p.I[k] = 10
        p.A[k] = P
    p.X, p.lam, p.xdtype, p.prec, p.error_mode = P, P, 0, 1, 0
    assert L.cpqr_als_work(ctypes.byref(p)) == 0
    w = L.cpqr_als_ne_work(ctypes.byref(p))
    # Gram matrices (3 x 16), S and its factor, Y (10 x 16), M (10 x 4) at least
    assert w >= 8 * (48 + 32 + 160 + 40)
    p.A[1] = None
    assert L.cpqr_als_ne_work(ctypes.byref(p)) == 0
    assert L.cpqr_als_ne_init(ctypes.byref(p), P, 1 << 30, None) == -1
    p.A[1] = P
    assert L.cpqr_als_ne_sweep(ctypes.byref(p), -1, None, P, 1 << 30, None) == -1
    assert L.cpqr_als_ne_sweep(ctypes.byref(p), 1, None, P, 16, None) == -4
    p.I[2] = 3
    assert L.cpqr_als_ne_init(ctypes.byref(p), P, 1 << 30, None) == -2


def test_workspace_queries(L):
    # up to 1024 rows: one node, no work buffer; 5000 x 16: five 1024-row
    # leaves (reflectors 1024 x 16 and T 16 x 16 each) under a root that
    # stacks their five 16 x 16 R factors
    assert L.cpqr_factor_qr_work(1000, 16) == 0
    assert L.cpqr_factor_qr_work(5000, 16) == 8 * (5 * 1024 * 16 + 5 * 256 + 5 * 256)
    assert L.cpqr_factor_qr_work(1000, 0) == 0
    assert L.cpqr_krp_qr_work(4, 32) >= 32768 * 32 * 8
    for n in range(3):
        w = L.cpqr_multittm_work(3, C._i64_array([1000, 1000, 1000]), n, 16, 1)
        assert 64e6 <= w < 200e6  # one 64 MB intermediate plus small pieces
    assert L.cpqr_apply_q0_work(200, 32768, 32) > 0
    assert L.cpqr_fit_direct_work(3, C._i64_array([50, 50, 50]), 5) > 0


def test_no_cpu_fallback():
    """The binding refuses host tensors instead of computing on the CPU."""
    import torch
    with pytest.raises(TypeError):
        C.cpqr_factor_qr(torch.zeros(8, 2, dtype=torch.float64))


def test_validation_batch_learned_dimtree(L):
    P = 4096
    # sweep: the dimension-tree split must be -1, 0 or in [1, N-1]
    p = C.Problem()
    p.N, p.R = 3, 4
    for k in range(3):
        p.I[k] = 10
        p.A[k] = p.Q[k] = p.Rf[k] = P
    p.X, p.lam, p.xdtype, p.prec, p.error_mode = P, P, 0, 1, 0
    for ok in (-1, 0, 1, 2):
        p.dimtree = ok
        assert L.cpqr_als_work(ctypes.byref(p)) > 0, ok
    for bad in (-2, 3, 7):
        p.dimtree = bad
        assert L.cpqr_als_work(ctypes.byref(p)) == 0, bad
    # batch: rank and mode-size limits
    items = (C.BatchItem * 1)()
    items[0].I[0], items[0].I[1], items[0].I[2] = 20, 30, 40
    items[0].R, items[0].X, items[0].lam = 4, P, P
    for k in range(3):
        items[0].A[k] = P
    assert L.cpqr_als_batch_work(items, 1) > 0
    items[0].R = 17
    assert L.cpqr_als_batch_work(items, 1) == 0
    assert L.cpqr_als_batch_prepare(items, 1, 0, P, 1 << 30, None) == -2
    items[0].R, items[0].I[1] = 4, 300
    assert L.cpqr_als_batch_prepare(items, 1, 0, P, 1 << 30, None) == -2
    assert L.cpqr_als_batch_run(None, 1, 1, 0, 0, None) == -4
    # sketch: sizes
    I = C._i64_array([256, 256, 256])
    J = (ctypes.c_int * 3)(64, 64, 64)
    assert L.cpqr_sketch3_work(I, J) > 0
    assert L.cpqr_sketch3_work(C._i64_array([100, 64, 64]), J) == 0
    assert L.cpqr_sketch3_work(I, (ctypes.c_int * 3)(64, 48, 64)) == 0
    Sp = (ctypes.c_void_p * 3)(P, P, P)
    assert L.cpqr_sketch3(I, P, J, Sp, P, None, P, 16, None) == -4
    assert L.cpqr_sketch3(I, None, J, Sp, P, None, P, 1 << 30, None) == -1
    # MLP: widths and batch multiples of 64, non-null weights
    net = C.Mlp(128, 64, 192, (ctypes.c_void_p * 3)(P, P, P), (ctypes.c_void_p * 3)(P, P, P))
    assert L.cpqr_mlp_work(ctypes.byref(net), 64) > 0
    assert L.cpqr_mlp_work(ctypes.byref(net), 32) == 0
    bad = C.Mlp(100, 64, 192, (ctypes.c_void_p * 3)(P, P, P), (ctypes.c_void_p * 3)(P, P, P))
    assert L.cpqr_mlp_work(ctypes.byref(bad), 64) == 0
    assert L.cpqr_mlp_forward(ctypes.byref(net), 64, None, P, P, P, P, 1 << 30, None) == -1
    assert L.cpqr_mlp_forward(ctypes.byref(bad), 64, P, P, P, P, P, 1 << 30, None) == -2
    # Kruskal loss: mode sizes <= 256, ranks <= 16, known loss kind, leading dimensions
    I3 = C._i64_array([32, 32, 32])
    assert L.cpqr_kruskal_loss_grad(1, C._i64_array([300, 4, 4]), 2, 2, P, 10000, P, 10000, 0, P, P, P, 1.0, None) == -2
    assert L.cpqr_kruskal_loss_grad(1, I3, 17, 2, P, 10000, P, 10000, 0, P, P, P, 1.0, None) == -2
    assert L.cpqr_kruskal_loss_grad(1, I3, 2, 2, P, 10000, P, 10000, 5, P, P, P, 1.0, None) == -1
    assert L.cpqr_kruskal_loss_grad(1, I3, 2, 2, P, 100, P, 10000, 0, P, P, P, 1.0, None) == -2
    # Adam and the bfloat16 conversion
    assert L.cpqr_adam(0, P, P, P, P, None, 1, 1e-3, 0.9, 0.999, 1e-8, None) == -1
    assert L.cpqr_adam(10, P, P, P, P, None, 0, 1e-3, 0.9, 0.999, 1e-8, None) == -1
    assert L.cpqr_to_bf16(None, 10, P, None) == -1
    assert L.cpqr_to_bf16(P, 0, P, None) == 0


def test_kruskal_validation_codes(L):
    """Kruskal-input entries (section 3.3.2): argument errors are caught
    before anything is enqueued."""
    P = 4096
    I = (C._i64 * 3)(5, 6, 7)
    V = (C._vp * 3)(P, P, P)
    Vnull = (C._vp * 3)(P, None, P)
    assert L.cpqr_kruskal_w_work(2, 4, 5) == 0
    assert L.cpqr_kruskal_w_work(3, 4, 5) > 0
    assert L.cpqr_kruskal_w(2, 0, 4, I, 5, P, V, V, P, P, P, 1 << 20, None) == -2
    assert L.cpqr_kruskal_w(3, 0, 4, I, 0, P, V, V, P, P, P, 1 << 20, None) == -2
    assert L.cpqr_kruskal_w(3, 0, 4, I, 5, None, V, V, P, P, P, 1 << 20, None) == -1
    assert L.cpqr_kruskal_w(3, 3, 4, I, 5, P, V, V, P, P, P, 1 << 20, None) == -1
    assert L.cpqr_kruskal_w(3, 0, 4, I, 5, P, Vnull, V, P, P, P, 1 << 20, None) == -1
    assert L.cpqr_kruskal_w(3, 0, 4, I, 5, P, V, V, P, P, None, 0, None) == -4
    assert L.cpqr_kruskal_mttkrp(3, 0, 33, I, 5, P, V, V, P, P, 1 << 20, None) == -2
    assert L.cpqr_kruskal_norm2(3, I, 5, P, V, None, P, 1 << 20, None) == -1
    assert L.cpqr_kruskal_full(3, I, 5, P, V, 7, P, P, 1 << 20, None) == -3
    big = (C._i64 * 2)(2, 5000000)
    assert L.cpqr_kruskal_full(2, big, 5, P, V, C.F64, P, P, 1 << 40, None) == -2
    p = C.Problem()
    p.N, p.R = 3, 4
    for k in range(3):
        p.I[k] = (5, 6, 7)[k]
        p.A[k] = p.Q[k] = p.Rf[k] = P
    p.lam = P
    p.xS = -1
    assert L.cpqr_als_work(ctypes.byref(p)) == 0
    p.xS, p.xmu = 5, P
    for k in range(3):
        p.xV[k] = P
    assert L.cpqr_als_work(ctypes.byref(p)) > 0  # no dense X needed
    p.error_mode = C.ERROR_DIRECT
    assert L.cpqr_als_work(ctypes.byref(p)) == 0  # the direct error needs X


def test_graph_validation_codes(L):
    P = 4096
    p = C.Problem()
    p.N, p.R = 3, 4
    for k in range(3):
        p.I[k] = 10
        p.A[k] = p.Q[k] = p.Rf[k] = P
    p.lam = p.X = P
    h = C._vp()
    assert L.cpqr_als_graph_create(ctypes.byref(p), 0, 1, P, P, 1 << 30, None) == -1
    assert L.cpqr_als_graph_create(ctypes.byref(p), 2, 1, P, P, 1 << 30, ctypes.byref(h)) == -1
    assert L.cpqr_als_graph_create(ctypes.byref(p), 0, 0, P, P, 1 << 30, ctypes.byref(h)) == -1
    assert L.cpqr_als_graph_create(ctypes.byref(p), 0, 1, P, None, 0, ctypes.byref(h)) == -4
    assert h.value is None
    assert L.cpqr_graph_launch(None, None) == -1
    assert L.cpqr_graph_destroy(None) == 0


def test_hosvd_validation_codes(L):
    P = 4096
    I = (C._i64 * 3)(10, 12, 14)
    Om = (C._vp * 3)(P, P, P)
    A = (C._vp * 3)(None, P, P)
    assert L.cpqr_hosvd_init_work(3, I, 4, C.PREC_F32) > 0
    assert L.cpqr_hosvd_init(3, I, C.F32, P, 4, Om, C.PREC_F32, 1, None, P, 1 << 30, None) == -1
    assert L.cpqr_hosvd_init(3, I, C.F32, P, 4, Om, C.PREC_F32, 3, A, P, 1 << 30, None) == -1
    assert L.cpqr_hosvd_init(3, I, C.F32, P, 4, Om, C.PREC_F32, 0, A, P, 1 << 30, None) == -1  # A[0] NULL
    assert L.cpqr_hosvd_init(3, I, C.F32, P, 33, Om, C.PREC_F32, 1, A, P, 1 << 30, None) == -2
    small = (C._i64 * 3)(10, 3, 14)
    assert L.cpqr_hosvd_init(3, small, C.F32, P, 4, Om, C.PREC_F32, 1, A, P, 1 << 30, None) == -2
    assert L.cpqr_hosvd_init(3, I, C.F32, P, 4, Om, C.PREC_F32, 1, A, None, 0, None) == -4
