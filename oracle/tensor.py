"""Tensor conventions and products, written out from their definitions.

Test infrastructure (see the package docstring): FP64, numpy only.

Index conventions (paper section 2.2, following Kolda and Bader):
  * A tensor is an ndarray of shape (I_1, ..., I_N) indexed (i_1, ..., i_N).
  * Mode-n unfolding X_(n) has I_n rows; the column of entry (i_1..i_N) is
    sum_{k != n} i_k * prod_{m < k, m != n} I_m (0-based), i.e. the
    lowest-numbered remaining mode varies fastest.  This is the ordering under
    which eq. (multittm) holds with the Kronecker factors listed from U_N down
    to U_1.
  * Kronecker product (section 2.2): (A kron B)[K*i + k, M*j + l] = A[i,j] B[k,l]
    for B of shape K x M (first factor's index varies slowest).
  * Khatri-Rao product (section 2.2): column-wise Kronecker product.
"""

import numpy as np


def kron(A, B):
    """Kronecker product A (x) B, section 2.2.  Library primitive np.kron,
    whose index convention the pin tests check against the definition."""
    return np.kron(np.asarray(A, dtype=np.float64), np.asarray(B, dtype=np.float64))


def khatri_rao(A, B):
    """Khatri-Rao product: column k is A[:, k] (x) B[:, k] (section 2.2)."""
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    if A.shape[1] != B.shape[1]:
        raise ValueError("Khatri-Rao factors need the same number of columns")
    cols = [np.kron(A[:, k], B[:, k]) for k in range(A.shape[1])]
    return np.stack(cols, axis=1)


def khatri_rao_list(mats):
    """Left-to-right Khatri-Rao product mats[0] (.) mats[1] (.) ... (.) mats[-1]."""
    out = np.asarray(mats[0], dtype=np.float64)
    for M in mats[1:]:
        out = khatri_rao(out, M)
    return out


def kron_list(mats):
    """Left-to-right Kronecker product mats[0] (x) ... (x) mats[-1]."""
    out = np.asarray(mats[0], dtype=np.float64)
    for M in mats[1:]:
        out = kron(out, M)
    return out


def hadamard_list(mats):
    """Elementwise (Hadamard) product of equally-shaped matrices (section 2.2)."""
    out = np.array(mats[0], dtype=np.float64)
    for M in mats[1:]:
        out = out * M
    return out


def unfold(X, n):
    """Mode-n matricization X_(n) (section 2.2), 0-based mode n.

    Rows are indexed by i_n; columns are the mode-n fibers ordered with the
    lowest-numbered remaining mode fastest.
    """
    X = np.asarray(X)
    moved = np.moveaxis(X, n, 0)
    return moved.reshape(X.shape[n], -1, order="F")


def fold(M, n, shape):
    """Inverse of :func:`unfold` for a tensor of the given full shape."""
    shape = tuple(int(s) for s in shape)
    rest = shape[:n] + shape[n + 1:]
    moved = np.asarray(M).reshape((shape[n],) + rest, order="F")
    return np.moveaxis(moved, 0, n)


def ttm(X, U, n):
    """n-mode product Y = X x_n U (section 2.2): Y_(n) = U X_(n).

    U has shape J x I_n; the result has I_n replaced by J.
    """
    U = np.asarray(U, dtype=np.float64)
    shape = list(X.shape)
    if U.shape[1] != shape[n]:
        raise ValueError("TTM: U has %d columns, mode %d has size %d" % (U.shape[1], n, shape[n]))
    Yn = U @ unfold(np.asarray(X, dtype=np.float64), n)
    shape[n] = U.shape[0]
    return fold(Yn, n, shape)


def multittm_order(shape, n):
    """The TTM order the oracle uses for the Multi-TTM of all modes except n:
    decreasing mode size, ties broken by ascending mode index (section 3.2,
    which orders the TTMs by decreasing dimension to minimise flops)."""
    modes = [k for k in range(len(shape)) if k != n]
    return sorted(modes, key=lambda k: (-shape[k], k))


def multittm(X, U, n, order=None):
    """Multi-TTM in every mode except n (section 2.2, eq. multittm):
    Y = X x_k U[k] for all k != n, applied one TTM at a time.

    ``U`` is a sequence indexed by mode (U[n] is ignored).  ``order`` is the
    sequence of modes to contract; by default :func:`multittm_order`.  The
    paper notes the TTMs may be applied in any order.
    """
    if order is None:
        order = multittm_order(X.shape, n)
    Y = np.asarray(X, dtype=np.float64)
    for k in order:
        Y = ttm(Y, U[k], k)
    return Y


def mttkrp(X, mats, n):
    """MTTKRP M_n = X_(n) Z_n with Z_n the Khatri-Rao product of all factors
    but the n-th, listed from mode N down to mode 1 (section 2.3, Alg. 1)."""
    N = X.ndim
    Z = khatri_rao_list([mats[k] for k in reversed(range(N)) if k != n])
    return unfold(np.asarray(X, dtype=np.float64), n) @ Z


def full(lam, mats):
    """Dense tensor of the Kruskal model [[lam; A_1..A_N]] (eq. cp):
    sum_r lam_r a_r^(1) o ... o a_r^(N), built through eq. (cp_mat) for
    mode 1: X_(1) = A_1 diag(lam) (A_N (.) ... (.) A_2)^T."""
    N = len(mats)
    shape = tuple(M.shape[0] for M in mats)
    A1 = np.asarray(mats[0], dtype=np.float64) * np.asarray(lam, dtype=np.float64)[None, :]
    if N == 1:
        return A1.sum(axis=1)
    Z = khatri_rao_list([mats[k] for k in reversed(range(1, N))])
    return fold(A1 @ Z.T, 0, shape)


def norm(X):
    """Frobenius norm, accumulated in float64."""
    X = np.asarray(X, dtype=np.float64)
    return float(np.sqrt(np.sum(X * X)))
