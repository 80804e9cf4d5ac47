"""Alg. 1 of the paper (CP-ALS with the normal equations, and CP-ALS-PINV),
the comparator for CP-ALS-QR.  FP64, step by step.

Test infrastructure (see the package docstring).

Mode update (section 2.3): S_n = Hadamard product of the Gram matrices
G_k = A_k^T A_k over k != n, M_n = X_(n) Z_n (MTTKRP), solve Ahat_n S_n = M_n
by Cholesky (CP-ALS) or with the pseudo-inverse of S_n (CP-ALS-PINV),
normalize, recompute G_n.  Error in the efficient form of section 3.3.1:
||X||^2 - 2 <M_N, Ahat_N> + <S_N, diag(lam) G_N diag(lam)>.
"""

import numpy as np
import scipy.linalg

from . import tensor as T


def default_rtol(R):
    """Relative cutoff of the pseudo-inverse: singular values of S_n at or
    below R * 2^-52 times the largest are dropped, the reading of MATLAB's
    pinv default (size times the spacing of doubles at the norm) that the
    SVD solve of CP-ALS-QR also takes."""
    return R * 2.0 ** -52


def mode_update(X, A, G, n, solver="chol", rtol=None):
    """One Alg. 1 mode update; updates A[n], G[n] in place.
    Returns (Ahat, lam, M, S)."""
    N = X.ndim
    S = T.hadamard_list([G[k] for k in range(N) if k != n])
    M = T.mttkrp(X, A, n)
    if solver == "chol":
        c = scipy.linalg.cho_factor(S, lower=False, check_finite=False)
        Ahat = scipy.linalg.cho_solve(c, M.T, check_finite=False).T
    elif solver == "pinv":
        if rtol is None or rtol < 0:
            rtol = default_rtol(S.shape[0])
        Ahat = M @ np.linalg.pinv(S, rcond=rtol)
    else:
        raise ValueError("solver must be 'chol' or 'pinv'")
    lam = np.sqrt(np.sum(Ahat * Ahat, axis=0))
    safe = np.where(lam > 0, lam, 1.0)
    A[n] = Ahat / safe[None, :]
    G[n] = A[n].T @ A[n]
    return Ahat, lam, M, S


def cp_als(X, A_init, maxiters=25, tol=0.0, solver="chol", error="efficient", rtol=None):
    """CP-ALS / CP-ALS-PINV (Alg. 1).  Returns (lam, A, relerr history)."""
    X = np.asarray(X, dtype=np.float64)
    N = X.ndim
    A = [np.array(a, dtype=np.float64) for a in A_init]
    G = [a.T @ a for a in A]
    xnorm2 = float(np.sum(X * X))
    lam = np.ones(A[0].shape[1])
    hist = []
    for s in range(maxiters):
        for n in range(N):
            Ahat, lam, M, S = mode_update(X, A, G, n, solver=solver, rtol=rtol)
        if error == "efficient":
            ip = float(np.sum(M * Ahat))
            nn = float(np.sum(S * ((lam[:, None] * G[N - 1]) * lam[None, :])))
            rel = float(np.sqrt(max(xnorm2 - 2.0 * ip + nn, 0.0)) / np.sqrt(xnorm2))
        else:
            rel = T.norm(X - T.full(lam, A)) / np.sqrt(xnorm2)
        hist.append(rel)
        if s >= 1 and abs(hist[-2] - hist[-1]) < tol:
            break
    return lam, A, hist
