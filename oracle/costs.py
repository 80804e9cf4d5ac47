"""Flop model of one CP-ALS-QR mode update (section 3.2).

Test infrastructure (see the package docstring).  These counts give the
algorithmic flops that roofline figures divide by measured time.
"""

from . import tensor as T


def ttm_sequence_flops(shape, n, R, order=None):
    """Flops of the Multi-TTM of all modes but n done as a sequence of TTMs,
    each contracting one mode of the current tensor of size D (with that
    mode's size D_k) into R: 2 * R * prod(D) per TTM (section 3.2)."""
    if order is None:
        order = T.multittm_order(shape, n)
    dims = [int(s) for s in shape]
    total = 0
    for k in order:
        size = 1
        for d in dims:
            size *= d
        total += 2 * R * size
        dims[k] = R
    return total


def ttm_cost_closed_form(shape, n, R):
    """eq. (TTMcost) for the decreasing-size order: 2 prod(I) R (1 + R/I_(1)
    + R^2/(I_(1) I_(2)) + ...), with I_(j) the j-th largest size among the
    contracted modes and N-1 terms in the bracket."""
    dims = sorted([int(shape[k]) for k in range(len(shape)) if k != n], reverse=True)
    prod_all = 1
    for s in shape:
        prod_all *= int(s)
    bracket = 0.0
    denom = 1
    for j in range(len(dims)):
        bracket += R ** j / denom
        denom *= dims[j]
    return 2.0 * prod_all * R * bracket


def krp_qr_flops(N, R):
    """eq. (QRcost): 4 R^{N+1}, leading order, Q_0 formed explicitly."""
    return 4 * R ** (N + 1)
