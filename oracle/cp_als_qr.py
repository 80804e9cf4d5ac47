"""Alg. 2 of the paper (CP-ALS-QR and CP-ALS-QR-SVD), step by step, in FP64.

Test infrastructure (see the package docstring).

Each mode update solves the least-squares problem of eq. (ls_n),
    min over Ahat_n of || X_(n) - Ahat_n Z_n^T ||_F,
through the QR of Z_n assembled from per-factor QRs (section 3.1):
    A_k = Q_k R_k,   V_n = R_N (.) ... (.) R_{n+1} (.) R_{n-1} (.) ... (.) R_1,
    V_n = Q_0 R_0,   Z_n = (Q_N (x) ... (x) Q_1) Q_0 R_0          (eq. Z_qr)
then the Multi-TTM Y = X x_{k != n} Q_k^T, W_n = Y_(n) Q_0 and the solve
Ahat_n R_0^T = W_n by substitution (CP-ALS-QR) or through the SVD of R_0 with
a pseudo-inverse (CP-ALS-QR-SVD), eq. (ls-qr-step), (ls-qr-ttm-step),
(ls-qr-q0-step).  Modes are 0-based here (mode n of the paper is n-1).

Readings of points the paper leaves open (each is listed in the design notes):
  * Q_n, R_n are recomputed from the *normalized* A_n (the error formula of
    section 3.3.1 calls R_N the triangular factor of the QR of A_N).
  * Default SVD truncation: keep sigma_i > rtol * sigma_1 with
    rtol = R * 2^-52 (the paper gives no threshold; this is the usual
    pseudo-inverse default).
  * Termination: after each full sweep, stop when |relerr_{s-1} - relerr_s|
    < tol, or after maxiters sweeps.
"""

import numpy as np
import scipy.linalg

from . import tensor as T

EPS = float(np.finfo(np.float64).eps)

# status bits, mirrored by nothing: the GPU library defines its own
SINGULAR_R0 = 1
NONFINITE = 2
RANK_TRUNCATED = 4


def factor_qr(A):
    """Compact (thin) QR of a factor matrix, A = Q R (Alg. 2, QR of the
    factor matrices).  Library primitive: LAPACK Householder QR."""
    Q, R = np.linalg.qr(np.asarray(A, dtype=np.float64), mode="reduced")
    return Q, R


def krp_of_r(Rs, n):
    """V_n = R_N (.) ... (.) R_{n+1} (.) R_{n-1} (.) ... (.) R_1 (section 3.1).

    ``Rs`` is indexed by mode; Rs[n] is ignored.  Row index of V_n has the
    lowest remaining mode fastest, matching the column order of Y_(n).
    """
    N = len(Rs)
    return T.khatri_rao_list([Rs[k] for k in reversed(range(N)) if k != n])


def krp_qr(Rs, n):
    """Compact QR V_n = Q_0 R_0 with Q_0 formed explicitly (Alg. 2; section
    3.2 prices it at 4 R^{N+1} with Q_0 explicit)."""
    V = krp_of_r(Rs, n)
    Q0, R0 = np.linalg.qr(V, mode="reduced")
    return Q0, R0


def multittm_unfolded(X, Qs, n, order=None):
    """Y_(n) for Y = X x_1 Q_1^T ... x_{n-1} Q_{n-1}^T x_{n+1} Q_{n+1}^T ...
    x_N Q_N^T (Alg. 2 Multi-TTM step; eq. multittm with U_k = Q_k^T).
    Shape I_n x R^{N-1}."""
    U = [None if Q is None else np.asarray(Q, dtype=np.float64).T for Q in Qs]
    Y = T.multittm(X, U, n, order=order)
    return T.unfold(Y, n)


def apply_q0(Yn, Q0):
    """W_n = Y_(n) Q_0 (Alg. 2, eq. ls-qr-q0-step)."""
    return np.asarray(Yn, dtype=np.float64) @ np.asarray(Q0, dtype=np.float64)


def solve_qr(W, R0):
    """Ahat R_0^T = W by substitution (CP-ALS-QR).  Equivalent to the upper
    triangular system R_0 Ahat^T = W^T.  Returns (Ahat, status)."""
    status = 0
    d = np.diag(R0)
    if np.any(d == 0) or not np.all(np.isfinite(d)):
        status |= SINGULAR_R0
    with np.errstate(all="ignore"):
        At = scipy.linalg.solve_triangular(R0, np.asarray(W, dtype=np.float64).T,
                                           lower=False, check_finite=False)
    Ahat = At.T
    if not np.all(np.isfinite(Ahat)):
        status |= NONFINITE
    return Ahat, status


def default_rtol(R):
    """Relative singular-value cutoff used when the caller gives none."""
    return R * EPS


def solve_svd(W, R0, rtol=None):
    """CP-ALS-QR-SVD solve (section 3.1): R_0 = U S V^T and
    Ahat = W U S^+ V^T, where S^+ inverts the singular values above
    rtol * sigma_max and zeroes the rest.  Returns (Ahat, kept, status)."""
    R = R0.shape[0]
    if rtol is None or rtol < 0:
        rtol = default_rtol(R)
    U, s, Vt = np.linalg.svd(np.asarray(R0, dtype=np.float64))
    tau = rtol * (s[0] if s.size else 0.0)
    keep = s > tau
    kept = int(np.count_nonzero(keep))
    sinv = np.zeros_like(s)
    sinv[keep] = 1.0 / s[keep]
    Ahat = np.asarray(W, dtype=np.float64) @ (U * sinv[None, :]) @ Vt
    status = RANK_TRUNCATED if kept < R else 0
    if not np.all(np.isfinite(Ahat)):
        status |= NONFINITE
    return Ahat, kept, status


def normalize(Ahat):
    """Column 2-norms lambda_r and A = Ahat diag(lambda)^{-1} (Alg. 2,
    normalization step; eq. cp asks for unit columns).  A zero column stays
    zero with lambda_r = 0."""
    lam = np.sqrt(np.sum(Ahat * Ahat, axis=0))
    safe = np.where(lam > 0, lam, 1.0)
    return Ahat / safe[None, :], lam


def error_efficient(xnorm2, W, Ahat, R0, lam, RN):
    """Relative error from quantities of the last mode update (section 3.3.1):
    <X, Xhat> = <W_N, Ahat_N R_0^T>,
    ||Xhat||^2 = <R_0^T R_0, diag(lam) R_N^T R_N diag(lam)>,
    relerr = sqrt(max(||X||^2 - 2<X,Xhat> + ||Xhat||^2, 0)) / ||X||."""
    ip = float(np.sum(W * (Ahat @ R0.T)))
    G0 = R0.T @ R0
    GN = (lam[:, None] * (RN.T @ RN)) * lam[None, :]
    nn = float(np.sum(G0 * GN))
    r2 = xnorm2 - 2.0 * ip + nn
    return float(np.sqrt(max(r2, 0.0)) / np.sqrt(xnorm2))


def error_direct(X, lam, A):
    """Relative error ||X - [[lam; A]]|| / ||X|| with the model formed
    explicitly (section 3.3.1, the accurate form)."""
    X = np.asarray(X, dtype=np.float64)
    Xhat = T.full(lam, A)
    return T.norm(X - Xhat) / T.norm(X)


class State:
    """ALS state: normalized factors, their thin QRs and the weights."""

    def __init__(self, A, Q, R, lam):
        self.A, self.Q, self.R, self.lam = A, Q, R, lam

    def copy(self):
        cp = lambda L: [None if x is None else np.array(x) for x in L]
        return State(cp(self.A), cp(self.Q), cp(self.R), np.array(self.lam))


def init_state(A_init):
    """Alg. 2 set-up: take the initial factors for modes 2..N (the mode-1
    initial factor is not used) and compute their compact QRs."""
    N = len(A_init)
    A = [None] + [np.array(A_init[k], dtype=np.float64) for k in range(1, N)]
    Q, R = [None] * N, [None] * N
    for k in range(1, N):
        Q[k], R[k] = factor_qr(A[k])
    Rk = A_init[1].shape[1]
    return State(A, Q, R, np.ones(Rk))


def mode_update(X, st, n, solver="qr", rtol=None, order=None):
    """One mode-n update of Alg. 2, in the paper's order.  Updates ``st`` in
    place and returns the intermediates (for step-by-step comparison)."""
    Q0, R0 = krp_qr(st.R, n)
    Yn = multittm_unfolded(X, st.Q, n, order=order)
    W = apply_q0(Yn, Q0)
    kept = R0.shape[0]
    if solver == "qr":
        Ahat, status = solve_qr(W, R0)
    elif solver == "svd":
        Ahat, kept, status = solve_svd(W, R0, rtol)
    else:
        raise ValueError("solver must be 'qr' or 'svd'")
    A, lam = normalize(Ahat)
    st.A[n], st.lam = A, lam
    st.Q[n], st.R[n] = factor_qr(A)
    return dict(Q0=Q0, R0=R0, Yn=Yn, W=W, Ahat=Ahat, kept=kept, status=status)


def sweep(X, st, solver="qr", rtol=None, error="efficient", xnorm2=None):
    """One full sweep over modes 1..N followed by the error (Alg. 2 inner
    loop).  Returns (relerr, per-mode intermediates)."""
    X = np.asarray(X, dtype=np.float64)
    if xnorm2 is None:
        xnorm2 = float(np.sum(X * X))
    inter = []
    for n in range(X.ndim):
        inter.append(mode_update(X, st, n, solver=solver, rtol=rtol))
    last = inter[-1]
    if error == "efficient":
        rel = error_efficient(xnorm2, last["W"], last["Ahat"], last["R0"], st.lam, st.R[X.ndim - 1])
    elif error == "direct":
        rel = error_direct(X, st.lam, st.A)
    else:
        raise ValueError("error must be 'efficient' or 'direct'")
    return rel, inter


def cp_als_qr(X, A_init, maxiters=25, tol=0.0, solver="qr", rtol=None, error="efficient"):
    """CP-ALS-QR / CP-ALS-QR-SVD (Alg. 2).  Returns (lam, A, relerr history)."""
    X = np.asarray(X, dtype=np.float64)
    st = init_state(A_init)
    xnorm2 = float(np.sum(X * X))
    hist = []
    for s in range(maxiters):
        rel, _ = sweep(X, st, solver=solver, rtol=rtol, error=error, xnorm2=xnorm2)
        hist.append(rel)
        if s >= 1 and abs(hist[-2] - hist[-1]) < tol:
            break
    return st.lam, st.A, hist
