"""ctypes binding of libcpqr (include/cpqr.h).

Argument marshalling only: every step of CP-ALS-QR runs in the library's HIP
kernels.  PyTorch supplies device memory and the current stream.  The
functions keep the C names.

Layout conventions for torch tensors:
  * a column-major I x R matrix is a 2-D tensor of shape (I, R) with strides
    (1, I) -- see :func:`colmajor`;
  * a column-major tensor of sizes (I_1, ..., I_N) has strides
    (1, I_1, I_1 I_2, ...) -- see :func:`colmajor`.
There is no CPU fallback: if the library is missing, or a tensor is not on a
GPU, the call raises.
"""

import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.environ.get("CPQR_LIB") or os.path.join(HERE, "libcpqr.so")

MAX_MODES = 10
MAX_RANK = 32

F32, F64 = 0, 1
PREC_F64, PREC_F32, PREC_BF16X2, PREC_BF16 = 0, 1, 2, 3
STATUS_SINGULAR, STATUS_NONFINITE, STATUS_TRUNCATED, STATUS_ZERO_COLUMN = 1, 2, 4, 8
STATUS_ILL_CONDITIONED = 16
ERROR_EFFICIENT, ERROR_DIRECT, ERROR_NONE = 0, 1, 2
NPHASES = 8
PHASES = ["multittm", "ttm_first", "factor_qr", "q0", "apply_q0", "solve", "error", "ttm_stream_m"]

PREC_NAMES = {"f64": PREC_F64, "f32": PREC_F32, "bf16x2": PREC_BF16X2, "bf16": PREC_BF16}

_i64 = ctypes.c_int64
_vp = ctypes.c_void_p
_sz = ctypes.c_size_t


class CpqrError(RuntimeError):
    """A libcpqr entry point returned an error code."""

    def __init__(self, name, code, msg):
        super().__init__("%s failed (%d): %s" % (name, code, msg))
        self.code = code


class Problem(ctypes.Structure):
    """Mirror of ``cpqr_problem``."""
    _fields_ = [
        ("N", ctypes.c_int), ("R", ctypes.c_int),
        ("I", _i64 * MAX_MODES),
        ("xdtype", ctypes.c_int), ("X", _vp),
        ("A", _vp * MAX_MODES), ("Q", _vp * MAX_MODES), ("Rf", _vp * MAX_MODES),
        ("lam", _vp),
        ("prec", ctypes.c_int), ("use_svd", ctypes.c_int), ("rtol", ctypes.c_double),
        ("error_mode", ctypes.c_int), ("status", _vp), ("dimtree", ctypes.c_int), ("krp_chain", ctypes.c_int),
        ("xS", ctypes.c_int), ("xmu", _vp), ("xV", _vp * MAX_MODES),
    ]


class BatchItem(ctypes.Structure):
    """Mirror of ``cpqr_batch_item``."""
    _fields_ = [
        ("I", _i64 * 3), ("R", ctypes.c_int), ("X", _vp), ("A", _vp * 3), ("lam", _vp), ("relerr", _vp),
    ]


class Mlp(ctypes.Structure):
    """Mirror of ``cpqr_mlp``."""
    _fields_ = [("din", ctypes.c_int), ("hidden", ctypes.c_int), ("dout", ctypes.c_int),
                ("W", _vp * 3), ("b", _vp * 3)]


_lib = None

_SIGS = {
    "cpqr_last_error": (ctypes.c_char_p, []),
    "cpqr_version": (ctypes.c_int, []),
    "cpqr_factor_qr_work": (_sz, [_i64, ctypes.c_int]),
    "cpqr_factor_qr": (ctypes.c_int, [_i64, ctypes.c_int, _vp, _i64, _vp, _i64, _vp, _i64, _vp, _sz, _vp]),
    "cpqr_krp_qr_work": (_sz, [ctypes.c_int, ctypes.c_int]),
    "cpqr_krp_qr": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(_vp), _i64,
                                   _vp, _vp, _vp, _sz, _vp]),
    "cpqr_multittm_work": (_sz, [ctypes.c_int, ctypes.POINTER(_i64), ctypes.c_int, ctypes.c_int, ctypes.c_int]),
    "cpqr_multittm": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(_i64), ctypes.c_int, _vp, ctypes.c_int,
                                     ctypes.c_int, ctypes.POINTER(_vp), ctypes.c_int, _vp, _vp, _sz, _vp]),
    "cpqr_multittm_noalloc": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(_i64), ctypes.c_int, _vp, ctypes.c_int,
                                             ctypes.c_int, ctypes.POINTER(_vp), ctypes.c_int, _vp, _vp]),
    "cpqr_krp_qr_chain_work": (_sz, [ctypes.c_int, ctypes.c_int]),
    "cpqr_krp_qr_chain": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(_vp), _i64,
                                         _vp, _vp, _vp, _sz, _vp]),
    "cpqr_expand_q0_work": (_sz, [ctypes.c_int, ctypes.c_int]),
    "cpqr_expand_q0": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, _vp, _vp, _vp, _sz, _vp]),
    "cpqr_hosvd_init_work": (_sz, [ctypes.c_int, ctypes.POINTER(_i64), ctypes.c_int, ctypes.c_int]),
    "cpqr_hosvd_init": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(_i64), ctypes.c_int, _vp, ctypes.c_int,
                                       ctypes.POINTER(_vp), ctypes.c_int, ctypes.c_int, ctypes.POINTER(_vp), _vp, _sz,
                                       _vp]),
    "cpqr_kruskal_w_work": (_sz, [ctypes.c_int, ctypes.c_int, ctypes.c_int]),
    "cpqr_kruskal_w": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(_i64), ctypes.c_int,
                                      _vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp), _vp, _vp, _vp, _sz, _vp]),
    "cpqr_kruskal_mttkrp_work": (_sz, [ctypes.c_int, ctypes.c_int, ctypes.c_int]),
    "cpqr_kruskal_mttkrp": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(_i64),
                                           ctypes.c_int, _vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp), _vp, _vp,
                                           _sz, _vp]),
    "cpqr_kruskal_norm2_work": (_sz, [ctypes.c_int]),
    "cpqr_kruskal_norm2": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(_i64), ctypes.c_int, _vp,
                                          ctypes.POINTER(_vp), _vp, _vp, _sz, _vp]),
    "cpqr_kruskal_full_work": (_sz, [ctypes.c_int, ctypes.POINTER(_i64), ctypes.c_int]),
    "cpqr_kruskal_full": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(_i64), ctypes.c_int, _vp,
                                         ctypes.POINTER(_vp), ctypes.c_int, _vp, _vp, _sz, _vp]),
    "cpqr_apply_q0_chain_work": (_sz, [_i64, ctypes.c_int, ctypes.c_int]),
    "cpqr_apply_q0_chain": (ctypes.c_int, [_i64, ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp, _vp, _vp, _vp, _sz,
                                           _vp]),
    "cpqr_apply_q0_work": (_sz, [_i64, _i64, ctypes.c_int]),
    "cpqr_apply_q0": (ctypes.c_int, [_i64, _i64, ctypes.c_int, ctypes.c_int, _vp, _vp, _vp, _vp, _sz, _vp]),
    "cpqr_solve_rsvd_work": (_sz, [_i64, ctypes.c_int]),
    "cpqr_solve_rsvd": (ctypes.c_int, [_i64, ctypes.c_int, _vp, _vp, ctypes.c_int, ctypes.c_double, _vp, _vp,
                                       _vp, _vp, _sz, _vp]),
    "cpqr_fit_direct_work": (_sz, [ctypes.c_int, ctypes.POINTER(_i64), ctypes.c_int]),
    "cpqr_fit_direct": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(_i64), ctypes.c_int, _vp, ctypes.c_int, _vp,
                                       ctypes.POINTER(_vp), _vp, _vp, _sz, _vp]),
    "cpqr_als_work": (_sz, [ctypes.POINTER(Problem)]),
    "cpqr_als_init": (ctypes.c_int, [ctypes.POINTER(Problem), _vp, _sz, _vp]),
    "cpqr_als_sweep": (ctypes.c_int, [ctypes.POINTER(Problem), ctypes.c_int, _vp, _vp, _sz, _vp]),
    "cpqr_als_graph_create": (ctypes.c_int, [ctypes.POINTER(Problem), ctypes.c_int, ctypes.c_int, _vp, _vp, _sz,
                                             ctypes.POINTER(_vp)]),
    "cpqr_graph_launch": (ctypes.c_int, [_vp, _vp]),
    "cpqr_graph_destroy": (ctypes.c_int, [_vp]),
    "cpqr_als_ne_work": (_sz, [ctypes.POINTER(Problem)]),
    "cpqr_als_ne_init": (ctypes.c_int, [ctypes.POINTER(Problem), _vp, _sz, _vp]),
    "cpqr_als_ne_sweep": (ctypes.c_int, [ctypes.POINTER(Problem), ctypes.c_int, _vp, _vp, _sz, _vp]),
    "cpqr_als_batch_work": (_sz, [ctypes.POINTER(BatchItem), ctypes.c_int]),
    "cpqr_als_batch_prepare": (ctypes.c_int, [ctypes.POINTER(BatchItem), ctypes.c_int, ctypes.c_int, _vp, _sz, _vp]),
    "cpqr_als_batch_run": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp]),
    "cpqr_als_batch_graph": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp]),
    "cpqr_als_batch_config": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                             ctypes.POINTER(ctypes.c_int)]),
    "cpqr_sketch3_work": (_sz, [ctypes.POINTER(_i64), ctypes.POINTER(ctypes.c_int)]),
    "cpqr_sketch3": (ctypes.c_int, [ctypes.POINTER(_i64), _vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(_vp),
                                    _vp, _vp, _vp, _sz, _vp]),
    "cpqr_mlp_work": (_sz, [ctypes.POINTER(Mlp), ctypes.c_int]),
    "cpqr_mlp_forward": (ctypes.c_int, [ctypes.POINTER(Mlp), ctypes.c_int, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "cpqr_mlp_backward": (ctypes.c_int, [ctypes.POINTER(Mlp), ctypes.c_int, _vp, _vp, _vp, _vp, _vp,
                                         ctypes.POINTER(_vp), ctypes.POINTER(_vp), _vp, _sz, _vp]),
    "cpqr_kruskal_loss_grad": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(_i64), ctypes.c_int, ctypes.c_int, _vp,
                                              _i64, _vp, _i64, ctypes.c_int, _vp, _vp, _vp, ctypes.c_float, _vp]),
    "cpqr_adam": (ctypes.c_int, [_i64, _vp, _vp, _vp, _vp, _vp, ctypes.c_int, ctypes.c_float, ctypes.c_float,
                                 ctypes.c_float, ctypes.c_float, _vp]),
    "cpqr_to_bf16": (ctypes.c_int, [_vp, _i64, _vp, _vp]),
    "cpqr_timing_enable": (ctypes.c_int, [ctypes.c_int]),
    "cpqr_timing_reset": (ctypes.c_int, []),
    "cpqr_timing_select": (ctypes.c_int, [ctypes.c_uint]),
    "cpqr_timing_read": (ctypes.c_int, [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_i64), ctypes.c_int]),
}

EXPORTED = sorted(_SIGS)


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIBPATH):
            raise RuntimeError("libcpqr.so is not built (expected at %s); run __graft_entry__.build()" % LIBPATH)
        L = ctypes.CDLL(LIBPATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _call(name, *args):
    rc = getattr(lib(), name)(*args)
    if rc != 0:
        raise CpqrError(name, rc, lib().cpqr_last_error().decode())
    return rc


def _stream():
    return _vp(torch.cuda.current_stream().cuda_stream)


def _dev(t, what):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA (HIP) tensor" % what)
    return t


def _work(nbytes, device):
    """Scratch buffer of at least nbytes, 256-byte aligned; returns (keepalive, ptr)."""
    if nbytes == 0:
        return None, None
    buf = torch.empty(int(nbytes) + 256, dtype=torch.uint8, device=device)
    p = buf.data_ptr()
    return buf, p + ((-p) % 256)


def colmajor(x):
    """Same values, column-major strides (first index fastest)."""
    nd = x.dim()
    perm = list(reversed(range(nd)))
    return x.permute(perm).contiguous().permute(perm)


def empty_colmajor(shape, dtype, device):
    rev = list(reversed(shape))
    perm = list(reversed(range(len(shape))))
    return torch.empty(rev, dtype=dtype, device=device).permute(perm)


def _check_colmajor(x, what):
    exp = 1
    for d in range(x.dim()):
        if x.shape[d] > 1 and x.stride(d) != exp:
            raise ValueError("%s must be column-major (first index fastest)" % what)
        exp *= x.shape[d]


def _dtype_code(t):
    if t.dtype == torch.float32:
        return F32
    if t.dtype == torch.float64:
        return F64
    raise TypeError("tensor dtype must be float32 or float64")


def _ptr_array(ts):
    arr = (_vp * len(ts))()
    for i, t in enumerate(ts):
        arr[i] = None if t is None else t.data_ptr()
    return arr


def _i64_array(v):
    arr = (_i64 * len(v))()
    for i, x in enumerate(v):
        arr[i] = int(x)
    return arr


# ------------------------------------------------------------------ entry points

def cpqr_version():
    return lib().cpqr_version()


def cpqr_factor_qr(A):
    """Thin QR of an (I, R) column-major FP64 matrix -> (Q, Rk)."""
    _dev(A, "A")
    _check_colmajor(A, "A")
    I, R = A.shape
    Q = empty_colmajor((I, R), torch.float64, A.device)
    Rk = empty_colmajor((R, R), torch.float64, A.device)
    keep, w = _work(lib().cpqr_factor_qr_work(I, R), A.device)
    _call("cpqr_factor_qr", I, R, A.data_ptr(), I, Q.data_ptr(), I, Rk.data_ptr(), R, w,
          0 if keep is None else keep.numel() - 256, _stream())
    return Q, Rk


def cpqr_krp_qr(Rks, n):
    """QR of V_n = Khatri-Rao of the triangular factors (all but mode n).
    Rks: list of N (R, R) column-major FP64 tensors (entry n may be None)."""
    N = len(Rks)
    ref = next(r for r in Rks if r is not None)
    R = ref.shape[0]
    for k, r in enumerate(Rks):
        if k != n:
            _dev(r, "Rk")
            _check_colmajor(r, "Rk")
    K = R ** (N - 1)
    Q0 = empty_colmajor((K, R), torch.float64, ref.device)
    R0 = empty_colmajor((R, R), torch.float64, ref.device)
    keep, w = _work(lib().cpqr_krp_qr_work(N, R), ref.device)
    _call("cpqr_krp_qr", N, n, R, _ptr_array(Rks), R, Q0.data_ptr(), R0.data_ptr(), w,
          0 if keep is None else keep.numel() - 256, _stream())
    return Q0, R0


def cpqr_multittm(X, Qs, n, prec=PREC_F32):
    """Y_(n) of Y = X x_k Q_k^T (k != n).  X: column-major tensor (FP32 or
    FP64); Qs: list of (I_k, R) column-major FP64 (entry n may be None)."""
    _dev(X, "X")
    _check_colmajor(X, "X")
    prec = PREC_NAMES.get(prec, prec)
    N = X.dim()
    ref = next(q for q in Qs if q is not None)
    R = ref.shape[1]
    for k, q in enumerate(Qs):
        if k != n:
            _dev(q, "Q")
            _check_colmajor(q, "Q")
    I = _i64_array(X.shape)
    K = R ** (N - 1)
    ydt = torch.float64 if prec == PREC_F64 else torch.float32
    Y = empty_colmajor((X.shape[n], K), ydt, X.device)
    keep, w = _work(lib().cpqr_multittm_work(N, I, n, R, prec), X.device)
    _call("cpqr_multittm", N, I, _dtype_code(X), X.data_ptr(), n, R, _ptr_array(Qs), prec, Y.data_ptr(), w,
          0 if keep is None else keep.numel() - 256, _stream())
    return Y


NOALLOC_SCRATCH_BYTES = 128 << 20


def cpqr_multittm_noalloc(X, Qs, n, prec=PREC_F32, Y=None):
    """cpqr_multittm without a workspace: the library's static per-device
    scratch (NOALLOC_SCRATCH_BYTES) holds the intermediates.  Y may be given
    (a column-major I_n x R^(N-1) tensor of the output type) so that the call
    allocates nothing at all."""
    _dev(X, "X")
    _check_colmajor(X, "X")
    prec = PREC_NAMES.get(prec, prec)
    N = X.dim()
    ref = next(q for q in Qs if q is not None)
    R = ref.shape[1]
    for k, q in enumerate(Qs):
        if k != n:
            _dev(q, "Q")
            _check_colmajor(q, "Q")
    ydt = torch.float64 if prec == PREC_F64 else torch.float32
    shape = (X.shape[n], R ** (N - 1))
    if Y is None:
        Y = empty_colmajor(shape, ydt, X.device)
    elif Y.dtype != ydt or tuple(Y.shape) != shape:
        raise ValueError("Y must be %s of shape %s" % (ydt, shape))
    _dev(Y, "Y")
    _check_colmajor(Y, "Y")
    _call("cpqr_multittm_noalloc", N, _i64_array(X.shape), _dtype_code(X), X.data_ptr(), n, R, _ptr_array(Qs), prec,
          Y.data_ptr(), _stream())
    return Y


def cpqr_krp_qr_chain(Rks, n):
    """Structured QR of V_n: (Qc, R0) with Qc the (N-2) R^2 x R factors
    Q_2..Q_{N-1} stacked along a leading axis (each column-major)."""
    N = len(Rks)
    ref = next(r for r in Rks if r is not None)
    R = ref.shape[0]
    for k, r in enumerate(Rks):
        if k != n:
            _dev(r, "Rk")
            _check_colmajor(r, "Rk")
    Qc = torch.empty((N - 2, R, R * R), dtype=torch.float64, device=ref.device).transpose(1, 2)
    R0 = empty_colmajor((R, R), torch.float64, ref.device)
    nbytes = lib().cpqr_krp_qr_chain_work(N, R)
    keep, w = _work(nbytes, ref.device)
    _call("cpqr_krp_qr_chain", N, n, R, _ptr_array(Rks), R, Qc.data_ptr(), R0.data_ptr(), w, nbytes, _stream())
    return Qc, R0


def cpqr_expand_q0(Qc, N):
    """Q_0 (R^{N-1} x R, column-major FP64) formed from cpqr_krp_qr_chain's
    factors."""
    _dev(Qc, "Qc")
    R = Qc.shape[2]
    Q0 = empty_colmajor((R ** (N - 1), R), torch.float64, Qc.device)
    nbytes = lib().cpqr_expand_q0_work(N, R)
    keep, w = _work(nbytes, Qc.device)
    _call("cpqr_expand_q0", N, R, Qc.data_ptr(), Q0.data_ptr(), w, nbytes, _stream())
    return Q0


def cpqr_hosvd_init(X, Omegas, R, prec=PREC_F32, k0=1):
    """Randomized HOSVD start: list over modes of I_k x R orthonormal bases
    (None below k0) from the test factors Omegas (device FP64, I_k x R)."""
    _dev(X, "X")
    _check_colmajor(X, "X")
    prec = PREC_NAMES.get(prec, prec)
    N = X.dim()
    for o in Omegas:
        _dev(o, "Omega")
        _check_colmajor(o, "Omega")
    A = [empty_colmajor((X.shape[k], R), torch.float64, X.device) if k >= k0 else None for k in range(N)]
    I = _i64_array(X.shape)
    nbytes = lib().cpqr_hosvd_init_work(N, I, R, prec)
    keep, w = _work(nbytes, X.device)
    _call("cpqr_hosvd_init", N, I, _dtype_code(X), X.data_ptr(), R, _ptr_array(Omegas), prec, int(k0), _ptr_array(A),
          w, nbytes, _stream())
    return A


def _kruskal_args(mu, V):
    _dev(mu, "mu")
    if mu.dtype != torch.float64 or mu.dim() != 1:
        raise ValueError("mu must be a 1-D FP64 tensor")
    S = mu.shape[0]
    for k, v in enumerate(V):
        _dev(v, "V[%d]" % k)
        _check_colmajor(v, "V[%d]" % k)
        if v.dtype != torch.float64 or v.dim() != 2 or v.shape[1] != S:
            raise ValueError("V[%d] must be an I_k x S FP64 matrix" % k)
    return len(V), S, _i64_array([v.shape[0] for v in V])


def cpqr_kruskal_w(mu, V, Qs, Qc, n):
    """W = Y_(n) Q_0 for the Kruskal input [[mu; V]] and Y = X x_{k != n} Q_k^T,
    with Q_0 given by cpqr_krp_qr_chain's factors."""
    N, S, I = _kruskal_args(mu, V)
    _dev(Qc, "Qc")
    R = Qc.shape[2]
    W = empty_colmajor((V[n].shape[0], R), torch.float64, mu.device)
    nbytes = lib().cpqr_kruskal_w_work(N, R, S)
    keep, w = _work(nbytes, mu.device)
    _call("cpqr_kruskal_w", N, n, R, I, S, mu.data_ptr(), _ptr_array(V), _ptr_array(Qs), Qc.data_ptr(),
          W.data_ptr(), w, nbytes, _stream())
    return W


def cpqr_kruskal_mttkrp(mu, V, As, n):
    """M = X_(n) Z_n for the Kruskal input [[mu; V]] (As[n] not read)."""
    N, S, I = _kruskal_args(mu, V)
    R = next(a for a in As if a is not None).shape[1]
    M = empty_colmajor((V[n].shape[0], R), torch.float64, mu.device)
    nbytes = lib().cpqr_kruskal_mttkrp_work(N, R, S)
    keep, w = _work(nbytes, mu.device)
    _call("cpqr_kruskal_mttkrp", N, n, R, I, S, mu.data_ptr(), _ptr_array(V), _ptr_array(As), M.data_ptr(), w,
          nbytes, _stream())
    return M


def cpqr_kruskal_norm2(mu, V):
    """||[[mu; V]]||^2 as a one-element device tensor."""
    N, S, I = _kruskal_args(mu, V)
    out = torch.empty(1, dtype=torch.float64, device=mu.device)
    nbytes = lib().cpqr_kruskal_norm2_work(S)
    keep, w = _work(nbytes, mu.device)
    _call("cpqr_kruskal_norm2", N, I, S, mu.data_ptr(), _ptr_array(V), out.data_ptr(), w, nbytes, _stream())
    return out


def cpqr_kruskal_full(mu, V, dtype=torch.float64):
    """The dense tensor of [[mu; V]] (column-major) in FP64 or FP32."""
    N, S, I = _kruskal_args(mu, V)
    X = empty_colmajor(tuple(v.shape[0] for v in V), dtype, mu.device)
    nbytes = lib().cpqr_kruskal_full_work(N, I, S)
    keep, w = _work(nbytes, mu.device)
    _call("cpqr_kruskal_full", N, I, S, mu.data_ptr(), _ptr_array(V), _dtype_code(X), X.data_ptr(), w, nbytes,
          _stream())
    return X


def cpqr_apply_q0_chain(Y, Qc, N):
    """W = Y_(n) Q_0 with Q_0 given by cpqr_krp_qr_chain's factors."""
    _dev(Y, "Y")
    _check_colmajor(Y, "Y")
    In = Y.shape[0]
    R = Qc.shape[2]
    W = empty_colmajor((In, R), torch.float64, Y.device)
    nbytes = lib().cpqr_apply_q0_chain_work(In, N, R)
    keep, w = _work(nbytes, Y.device)
    _call("cpqr_apply_q0_chain", In, N, R, _dtype_code(Y), Y.data_ptr(), Qc.data_ptr(), W.data_ptr(), w, nbytes,
          _stream())
    return W


def cpqr_apply_q0(Y, Q0):
    """W = Y_(n) Q_0 in FP64."""
    _dev(Y, "Y")
    _dev(Q0, "Q0")
    _check_colmajor(Y, "Y")
    _check_colmajor(Q0, "Q0")
    In, K = Y.shape
    R = Q0.shape[1]
    W = empty_colmajor((In, R), torch.float64, Y.device)
    keep, w = _work(lib().cpqr_apply_q0_work(In, K, R), Y.device)
    _call("cpqr_apply_q0", In, K, R, _dtype_code(Y), Y.data_ptr(), Q0.data_ptr(), W.data_ptr(), w,
          0 if keep is None else keep.numel() - 256, _stream())
    return W


def cpqr_solve_rsvd(W, R0, use_svd=False, rtol=-1.0, status=None):
    """Solve Ahat R_0^T = W (substitution or SVD) and normalize -> (A, lambda)."""
    _dev(W, "W")
    _dev(R0, "R0")
    _check_colmajor(W, "W")
    _check_colmajor(R0, "R0")
    In, R = W.shape
    A = empty_colmajor((In, R), torch.float64, W.device)
    lam = torch.empty(R, dtype=torch.float64, device=W.device)
    keep, w = _work(lib().cpqr_solve_rsvd_work(In, R), W.device)
    _call("cpqr_solve_rsvd", In, R, W.data_ptr(), R0.data_ptr(), int(bool(use_svd)), float(rtol), A.data_ptr(),
          lam.data_ptr(), None if status is None else status.data_ptr(), w,
          0 if keep is None else keep.numel() - 256, _stream())
    return A, lam


def cpqr_fit_direct(X, lam, As):
    """(||X - [[lam; A]]||^2, ||X||^2) as a 2-element FP64 device tensor."""
    _dev(X, "X")
    _check_colmajor(X, "X")
    N = X.dim()
    R = As[0].shape[1]
    I = _i64_array(X.shape)
    out = torch.empty(2, dtype=torch.float64, device=X.device)
    keep, w = _work(lib().cpqr_fit_direct_work(N, I, R), X.device)
    _call("cpqr_fit_direct", N, I, _dtype_code(X), X.data_ptr(), R, lam.data_ptr(), _ptr_array(As),
          out.data_ptr(), w, 0 if keep is None else keep.numel() - 256, _stream())
    return out


def _input_shape(X, kruskal):
    """(shape, device) of the input: the dense X, or the Kruskal factors."""
    if kruskal is not None:
        mu, V = kruskal
        _kruskal_args(mu, V)
        shape = tuple(v.shape[0] for v in V)
        if X is not None:
            _dev(X, "X")
            _check_colmajor(X, "X")
            if tuple(X.shape) != shape:
                raise ValueError("X and the Kruskal factors disagree on the shape")
        return shape, mu.device
    _dev(X, "X")
    _check_colmajor(X, "X")
    return tuple(X.shape), X.device


def _set_input(p, X, kruskal):
    """Fill the input fields of a Problem; returns what must stay alive."""
    if X is not None:
        p.xdtype = _dtype_code(X)
        p.X = X.data_ptr()
    if kruskal is None:
        return None
    mu, V = kruskal
    p.xS = mu.shape[0]
    p.xmu = mu.data_ptr()
    for k, v in enumerate(V):
        p.xV[k] = v.data_ptr()
    return (mu, list(V))


class AlsState:
    """Device buffers of one CP-ALS-QR problem, wired into ``cpqr_problem``."""

    def __init__(self, X, init, prec=PREC_F32, use_svd=False, rtol=-1.0, error_mode=ERROR_EFFICIENT, dimtree=-1,
                 krp_chain=-1, kruskal=None):
        """kruskal=(mu, V): the input is the Kruskal tensor [[mu; V]] (section
        3.3.2); X is then optional, the same tensor in dense form, read only
        by the direct error."""
        shape, dev = _input_shape(X, kruskal)
        prec = PREC_NAMES.get(prec, prec)
        N = len(shape)
        R = init[1].shape[1]
        self.X, self.N, self.R = X, N, R
        self.dev = dev
        self.A = [colmajor(torch.as_tensor(init[k], dtype=torch.float64).to(dev)) if k > 0 else
                  empty_colmajor((shape[0], R), torch.float64, dev) for k in range(N)]
        if N > 0:
            self.A[0].zero_()
        self.Q = [empty_colmajor((shape[k], R), torch.float64, dev) for k in range(N)]
        self.Rf = [empty_colmajor((R, R), torch.float64, dev) for k in range(N)]
        self.lam = torch.ones(R, dtype=torch.float64, device=dev)
        self.status = torch.zeros(1, dtype=torch.int32, device=dev)
        p = Problem()
        p.N, p.R = N, R
        for k in range(N):
            p.I[k] = shape[k]
            p.A[k] = self.A[k].data_ptr()
            p.Q[k] = self.Q[k].data_ptr()
            p.Rf[k] = self.Rf[k].data_ptr()
        self.kruskal = _set_input(p, X, kruskal)
        p.lam = self.lam.data_ptr()
        p.prec, p.use_svd, p.rtol, p.error_mode = prec, int(bool(use_svd)), float(rtol), error_mode
        p.dimtree = int(dimtree)
        p.krp_chain = int(krp_chain)
        p.status = self.status.data_ptr()
        self.p = p
        nbytes = lib().cpqr_als_work(ctypes.byref(p))
        if nbytes == 0:
            raise CpqrError("cpqr_als_work", -1, lib().cpqr_last_error().decode())
        self._wkeep, self._w = _work(nbytes, dev)
        self._wbytes = nbytes

    def init(self):
        _call("cpqr_als_init", ctypes.byref(self.p), self._w, self._wbytes, _stream())

    def sweep(self, nsweeps=1, relerr=None):
        """Run nsweeps sweeps; returns the device tensor of relative errors."""
        if relerr is None:
            relerr = torch.empty(nsweeps, dtype=torch.float64, device=self.dev)
        _call("cpqr_als_sweep", ctypes.byref(self.p), int(nsweeps), relerr.data_ptr(), self._w, self._wbytes,
              _stream())
        return relerr

    def graph(self, nsweeps):
        """nsweeps sweeps captured into a HIP graph (SweepGraph)."""
        return SweepGraph(self, 0, nsweeps)


class SweepGraph:
    """nsweeps sweeps of a state captured into one HIP graph
    (cpqr_als_graph_create); launch() replays them on the current stream and
    leaves the relative errors in ``relerr``.  The state must stay alive."""

    def __init__(self, state, algo, nsweeps):
        self.state = state
        self.relerr = torch.empty(int(nsweeps), dtype=torch.float64, device=state.dev)
        h = _vp()
        _call("cpqr_als_graph_create", ctypes.byref(state.p), int(algo), int(nsweeps), self.relerr.data_ptr(),
              state._w, state._wbytes, ctypes.byref(h))
        self.h = h

    def launch(self):
        _call("cpqr_graph_launch", self.h, _stream())
        return self.relerr

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value and _lib is not None:
            _lib.cpqr_graph_destroy(h)
            self.h = None


def cpqr_als_init(state):
    state.init()


def cpqr_als_sweep(state, nsweeps=1, relerr=None):
    return state.sweep(nsweeps, relerr)


def cp_als_qr(X, init, maxiters=25, tol=0.0, prec=PREC_F32, use_svd=False, rtol=-1.0,
              error_mode=ERROR_EFFICIENT, dimtree=-1, krp_chain=-1, kruskal=None):
    """Alg. 2 driven from the host: sweeps until |relerr change| < tol or
    maxiters (reads the error back after each sweep only when tol > 0)."""
    st = AlsState(X, init, prec=prec, use_svd=use_svd, rtol=rtol, error_mode=error_mode, dimtree=dimtree,
                  krp_chain=krp_chain, kruskal=kruskal)
    st.init()
    if tol <= 0:
        rel = st.sweep(maxiters)
        return st, rel.cpu().tolist()
    hist = []
    for s in range(maxiters):
        hist.append(float(st.sweep(1)[0].item()))
        if s >= 1 and abs(hist[-2] - hist[-1]) < tol:
            break
    return st, hist


class AlsNeState:
    """Device buffers of one CP-ALS problem (Alg. 1, normal equations or
    pseudo-inverse), wired into ``cpqr_problem`` for cpqr_als_ne_*; every
    init[k] is the start of A_k (A_0 only through its Gram matrix)."""

    def __init__(self, X, init, prec=PREC_F32, solver="chol", rtol=-1.0, error_mode=ERROR_EFFICIENT, dimtree=-1,
                 kruskal=None):
        shape, dev = _input_shape(X, kruskal)
        if solver not in ("chol", "pinv"):
            raise ValueError("solver must be 'chol' or 'pinv'")
        prec = PREC_NAMES.get(prec, prec)
        N = len(shape)
        R = init[1].shape[1]
        self.X, self.N, self.R = X, N, R
        self.dev = dev
        self.A = [colmajor(torch.as_tensor(init[k], dtype=torch.float64).to(dev)) for k in range(N)]
        self.lam = torch.ones(R, dtype=torch.float64, device=dev)
        self.status = torch.zeros(1, dtype=torch.int32, device=dev)
        p = Problem()
        p.N, p.R = N, R
        for k in range(N):
            p.I[k] = shape[k]
            p.A[k] = self.A[k].data_ptr()
        self.kruskal = _set_input(p, X, kruskal)
        p.lam = self.lam.data_ptr()
        p.prec, p.use_svd, p.rtol, p.error_mode = prec, int(solver == "pinv"), float(rtol), error_mode
        p.dimtree = int(dimtree)
        p.status = self.status.data_ptr()
        self.p = p
        nbytes = lib().cpqr_als_ne_work(ctypes.byref(p))
        if nbytes == 0:
            raise CpqrError("cpqr_als_ne_work", -1, lib().cpqr_last_error().decode())
        self._wkeep, self._w = _work(nbytes, dev)
        self._wbytes = nbytes

    def init(self):
        _call("cpqr_als_ne_init", ctypes.byref(self.p), self._w, self._wbytes, _stream())

    def sweep(self, nsweeps=1, relerr=None):
        """Run nsweeps sweeps; returns the device tensor of relative errors."""
        if relerr is None:
            relerr = torch.empty(nsweeps, dtype=torch.float64, device=self.dev)
        _call("cpqr_als_ne_sweep", ctypes.byref(self.p), int(nsweeps), relerr.data_ptr(), self._w, self._wbytes,
              _stream())
        return relerr

    def graph(self, nsweeps):
        """nsweeps sweeps captured into a HIP graph (SweepGraph)."""
        return SweepGraph(self, 1, nsweeps)


def cp_als(X, init, maxiters=25, tol=0.0, prec=PREC_F32, solver="chol", rtol=-1.0, error_mode=ERROR_EFFICIENT,
           dimtree=-1, kruskal=None):
    """Alg. 1 (CP-ALS, or CP-ALS-PINV with solver='pinv') driven from the
    host, with the same stopping rule as cp_als_qr."""
    st = AlsNeState(X, init, prec=prec, solver=solver, rtol=rtol, error_mode=error_mode, dimtree=dimtree,
                    kruskal=kruskal)
    st.init()
    if tol <= 0:
        rel = st.sweep(maxiters)
        return st, rel.cpu().tolist()
    hist = []
    for s in range(maxiters):
        hist.append(float(st.sweep(1)[0].item()))
        if s >= 1 and abs(hist[-2] - hist[-1]) < tol:
            break
    return st, hist


def cp_als_hybrid(X, init, maxiters=25, prec=PREC_F32, error_mode=ERROR_EFFICIENT, dimtree=-1, kruskal=None):
    """The robust solver the paper envisions (section 1, section 5): CP-ALS
    with the normal equations while they are well conditioned, then CP-ALS-QR.
    The status word is read after every sweep.

    * A Cholesky step that proves cond(S_n) > 1e4 (cond(Z_n) > 100): the
      sweep is kept and CP-ALS-QR continues from its factors.
    * A breakdown (a non-positive Cholesky pivot, or a non-finite factor):
      the sweep's factors are not usable, so it is discarded and
      CP-ALS-QR-SVD redoes it from the factors the sweep started from (a
      device copy taken before every normal-equations sweep); the
      pseudo-inverse solve is defined also when Z_n is rank deficient
      (section 3.1), which is what a breakdown signals.

    Returns (state, history, number of normal-equations sweeps kept)."""
    st = AlsNeState(X, init, prec=prec, solver="chol", error_mode=error_mode, dimtree=dimtree, kruskal=kruskal)
    st.init()
    hist = []
    start, use_svd = None, False
    for s in range(maxiters):
        before = [a.clone() for a in st.A]
        rel = float(st.sweep(1)[0].item())
        flags = int(st.status.item())
        if flags & (STATUS_SINGULAR | STATUS_NONFINITE):
            start, use_svd = before, True
            break
        hist.append(rel)
        if flags & STATUS_ILL_CONDITIONED:
            start = [a.clone() for a in st.A]
            break
    n_ne = len(hist)
    if start is None:
        return st, hist, n_ne
    qst = AlsState(X, start, prec=prec, use_svd=use_svd, error_mode=error_mode, dimtree=dimtree, kruskal=kruskal)
    qst.init()
    hist += qst.sweep(maxiters - n_ne).cpu().tolist()
    return qst, hist, n_ne


class AlsBatch:
    """Device buffers of a batch of 3-way FP32 tensors for cpqr_als_batch_*.

    tensors: list of column-major FP32 CUDA tensors; inits: list of lists of
    three (I_k, R) initial factors (entry 0 unused); nsweeps_max: length of
    each tensor's relative-error record."""

    def __init__(self, tensors, inits, nsweeps_max, autotune=False):
        n = len(tensors)
        nsweeps_max = max(1, int(nsweeps_max))
        self.nsweeps_max = nsweeps_max
        self.tensors = tensors
        self.A, self.lam, self.relerr = [], [], []
        arr = (BatchItem * n)()
        for b, X in enumerate(tensors):
            _dev(X, "X")
            _check_colmajor(X, "X")
            if X.dtype != torch.float32 or X.dim() != 3:
                raise TypeError("batch tensors must be 3-way float32")
            R = inits[b][1].shape[1]
            dev = X.device
            A = [empty_colmajor((X.shape[0], R), torch.float64, dev).zero_()] + [
                colmajor(torch.as_tensor(inits[b][k], dtype=torch.float64).to(dev)) for k in (1, 2)]
            lam = torch.ones(R, dtype=torch.float64, device=dev)
            rel = torch.zeros(nsweeps_max, dtype=torch.float64, device=dev)
            self.A.append(A)
            self.lam.append(lam)
            self.relerr.append(rel)
            it = arr[b]
            for k in range(3):
                it.I[k] = X.shape[k]
                it.A[k] = A[k].data_ptr()
            it.R, it.X, it.lam, it.relerr = R, X.data_ptr(), lam.data_ptr(), rel.data_ptr()
        self.items = arr
        self.n = n
        nbytes = lib().cpqr_als_batch_work(arr, n)
        if nbytes == 0:
            raise CpqrError("cpqr_als_batch_work", -1, "bad batch")
        self._wkeep, self._w = _work(nbytes, tensors[0].device)
        self._wbytes = nbytes
        _call("cpqr_als_batch_prepare", arr, n, int(bool(autotune)), self._w, self._wbytes, _stream())

    @property
    def config(self):
        """(tensor rows per lane, steps in flight, 0: the row steps take whole modes)."""
        c, u, r = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _call("cpqr_als_batch_config", self._w, ctypes.byref(c), ctypes.byref(u), ctypes.byref(r))
        return c.value, u.value, r.value

    def run(self, nsweeps, init=False, offset=0, variant=0, graph=False):
        if offset + nsweeps > self.nsweeps_max:
            raise ValueError("relative-error record holds %d sweeps" % self.nsweeps_max)
        name = "cpqr_als_batch_graph" if graph else "cpqr_als_batch_run"
        _call(name, self._w, int(nsweeps), int(bool(init)), int(offset), int(variant), _stream())


def cpqr_timing_enable(on=True):
    _call("cpqr_timing_enable", int(bool(on)))


def cpqr_timing_select(phases=None):
    """Record only the named phases (all when None)."""
    mask = 0xFFFFFFFF if phases is None else sum(1 << PHASES.index(p) for p in phases)
    _call("cpqr_timing_select", ctypes.c_uint(mask))


def cpqr_timing_reset():
    _call("cpqr_timing_reset")


def cpqr_timing_read():
    ms = (ctypes.c_double * NPHASES)()
    cnt = (_i64 * NPHASES)()
    _call("cpqr_timing_read", ms, cnt, NPHASES)
    return {PHASES[i]: (ms[i], cnt[i]) for i in range(NPHASES)}


# ---------------------------------------------------------------- learned init
def _ptr(t):
    return None if t is None else t.data_ptr()


def _contig(t, dtype, what):
    _dev(t, what)
    if t.dtype != dtype or not t.is_contiguous():
        raise TypeError("%s must be a contiguous %s tensor" % (what, dtype))
    return t


def cpqr_to_bf16(x):
    """bfloat16 copy of a contiguous FP32 tensor (returned as torch.bfloat16)."""
    _contig(x, torch.float32, "x")
    y = torch.empty(x.shape, dtype=torch.bfloat16, device=x.device)
    _call("cpqr_to_bf16", x.data_ptr(), x.numel(), y.data_ptr(), _stream())
    return y


def cpqr_sketch3(X, S_bf16, normalized=True):
    """Sketch of a column-major FP32 3-way tensor: returns (xs FP32 vector,
    xs scaled to unit root-mean-square as bfloat16, or None)."""
    _dev(X, "X")
    _check_colmajor(X, "X")
    I = (_i64 * 3)(*X.shape)
    J = (ctypes.c_int * 3)(*[int(s.shape[0]) for s in S_bf16])
    for k in range(3):
        _contig(S_bf16[k], torch.bfloat16, "S")
    Sp = (_vp * 3)(*[s.data_ptr() for s in S_bf16])
    n = J[0] * J[1] * J[2]
    xs = torch.empty(n, dtype=torch.float32, device=X.device)
    xb = torch.empty(n, dtype=torch.bfloat16, device=X.device) if normalized else None
    nbytes = lib().cpqr_sketch3_work(I, J)
    if nbytes == 0:
        raise CpqrError("cpqr_sketch3_work", -2, "unsupported sketch shape")
    keep, w = _work(nbytes, X.device)
    _call("cpqr_sketch3", I, X.data_ptr(), J, Sp, xs.data_ptr(), _ptr(xb), w, nbytes, _stream())
    return xs, xb


class MlpNet:
    """Device views of a three-layer MLP: W[l] bfloat16 (out, in) and b[l]
    FP32; the struct passed to cpqr_mlp_*."""

    def __init__(self, W_bf16, b_f32):
        self.W, self.b = W_bf16, b_f32
        for t in W_bf16:
            _contig(t, torch.bfloat16, "W")
        for t in b_f32:
            _contig(t, torch.float32, "b")
        self.din, self.hidden, self.dout = W_bf16[0].shape[1], W_bf16[0].shape[0], W_bf16[2].shape[0]
        self.c = Mlp(self.din, self.hidden, self.dout, (_vp * 3)(*[w.data_ptr() for w in W_bf16]),
                     (_vp * 3)(*[b.data_ptr() for b in b_f32]))
        self._wk = {}

    def work(self, batch, device):
        if batch not in self._wk:
            nbytes = lib().cpqr_mlp_work(ctypes.byref(self.c), batch)
            if nbytes == 0:
                raise CpqrError("cpqr_mlp_work", -2, "unsupported MLP or batch shape")
            self._wk[batch] = (nbytes,) + _work(nbytes, device)
        return self._wk[batch]

    def forward(self, x_bf16):
        _contig(x_bf16, torch.bfloat16, "x")
        B = x_bf16.shape[0]
        dev = x_bf16.device
        h1 = torch.empty(B, self.hidden, dtype=torch.bfloat16, device=dev)
        h2 = torch.empty(B, self.hidden, dtype=torch.bfloat16, device=dev)
        y = torch.empty(B, self.dout, dtype=torch.float32, device=dev)
        nbytes, keep, w = self.work(B, dev)
        _call("cpqr_mlp_forward", ctypes.byref(self.c), B, x_bf16.data_ptr(), h1.data_ptr(), h2.data_ptr(),
              y.data_ptr(), w, nbytes, _stream())
        return y, (x_bf16, h1, h2)

    def backward(self, cache, dy, dy_bf16, dW, db):
        x, h1, h2 = cache
        B = x.shape[0]
        nbytes, keep, w = self.work(B, x.device)
        _call("cpqr_mlp_backward", ctypes.byref(self.c), B, x.data_ptr(), h1.data_ptr(), h2.data_ptr(),
              dy.data_ptr(), dy_bf16.data_ptr(), (_vp * 3)(*[t.data_ptr() for t in dW]),
              (_vp * 3)(*[t.data_ptr() for t in db]), w, nbytes, _stream())


LOSS_DISTANCE, LOSS_COSINE = 0, 1


def cpqr_kruskal_loss_grad(y, target, I, R, Rt, scale=1.0, kind=LOSS_DISTANCE):
    """Per-sample Kruskal losses and scale * dL/dy (FP32 and bfloat16)."""
    _contig(y, torch.float32, "y")
    _contig(target, torch.float32, "target")
    B = y.shape[0]
    loss = torch.empty(B, dtype=torch.float32, device=y.device)
    dy = torch.empty_like(y)
    dyb = torch.empty(y.shape, dtype=torch.bfloat16, device=y.device)
    _call("cpqr_kruskal_loss_grad", B, (_i64 * 3)(*I), R, Rt, y.data_ptr(), y.shape[1], target.data_ptr(),
          target.shape[1], int(kind), loss.data_ptr(), dy.data_ptr(), dyb.data_ptr(), float(scale), _stream())
    return loss, dy, dyb


def cpqr_adam(w, g, m, v, w_bf16, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    for t, nm in ((w, "w"), (g, "g"), (m, "m"), (v, "v")):
        _contig(t, torch.float32, nm)
    if w_bf16 is not None:
        _contig(w_bf16, torch.bfloat16, "w_bf16")
    _call("cpqr_adam", w.numel(), w.data_ptr(), g.data_ptr(), m.data_ptr(), v.data_ptr(), _ptr(w_bf16), int(step),
          float(lr), float(beta1), float(beta2), float(eps), _stream())
