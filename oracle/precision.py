"""Reduced-precision forms of the Multi-TTM contraction, emulated on the CPU.

Test infrastructure (see the package docstring).

The GPU offers the first (dominant) Multi-TTM contraction in FP32, in plain
bfloat16, and in a split form where each FP32 operand x is written as
x = x_hi + x_lo with x_hi = bf16(x), x_lo = bf16(x - x_hi), and a product is
taken as x_hi*q_hi + x_hi*q_lo + x_lo*q_hi (the x_lo*q_lo term is dropped),
accumulated in FP32.  The paper works in double precision throughout; these
forms are the reduced-precision variants whose error the tests measure
against the FP64 oracle.  bfloat16 rounding here is written out at bit level
(round to nearest, ties to even), independently of any library.
"""

import numpy as np


def round_bf16(x):
    """Round float32 values to the nearest bfloat16 (ties to even), returned
    as float32.  NaN stays NaN; overflow rounds to infinity as in IEEE."""
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = x.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = (u + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)
    out = r.astype(np.uint32).view(np.float32).copy()
    nan = np.isnan(x)
    out[nan] = x[nan]
    return out


def split_bf16(x):
    """x (float32) -> (hi, lo), both bfloat16 values held in float32, with
    hi = bf16(x) and lo = bf16(x - hi), the difference taken in float32."""
    x = np.asarray(x, dtype=np.float32)
    hi = round_bf16(x)
    lo = round_bf16((x - hi).astype(np.float32))
    return hi, lo


def contract_split(Xm, Qm):
    """Reference value of a split-bfloat16 contraction Xm @ Qm: the three
    kept partial products summed exactly (in float64)."""
    xh, xl = split_bf16(Xm)
    qh, ql = split_bf16(Qm)
    f = lambda a: a.astype(np.float64)
    return f(xh) @ f(qh) + f(xh) @ f(ql) + f(xl) @ f(qh)


def contract_bf16(Xm, Qm):
    """Reference value of a plain bfloat16 contraction (operands rounded to
    bfloat16, products summed exactly in float64)."""
    return round_bf16(Xm).astype(np.float64) @ round_bf16(Qm).astype(np.float64)


def multittm_lowp(X, Qs, n, mode, order=None):
    """Multi-TTM in every mode but n (eq. multittm with U_k = Q_k^T) where each
    TTM's products are taken in a reduced-precision form ("bf16": operands
    rounded to bfloat16; "bf16x2": the three kept split products), summed
    exactly, and the intermediate tensor is stored in FP32 as the GPU stores
    it.  Returns Y_(n) in float64."""
    from . import tensor as T
    if order is None:
        order = T.multittm_order(X.shape, n)
    Y = np.asarray(X, dtype=np.float32)
    for k in order:
        Q = np.asarray(Qs[k], dtype=np.float64)
        Ym = T.unfold(Y, k).T.astype(np.float32)  # rows: other indices, cols: mode k
        Qf = Q.astype(np.float32)
        Z = contract_split(Ym, Qf) if mode == "bf16x2" else contract_bf16(Ym, Qf)
        shape = list(Y.shape)
        shape[k] = Q.shape[1]
        Y = T.fold(Z.T, k, shape).astype(np.float32)
    return T.unfold(Y, n).astype(np.float64)
