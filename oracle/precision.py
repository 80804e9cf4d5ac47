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
