"""CP-ALS-QR and CP-ALS on an input tensor given in Kruskal form (section
3.3.2), with the structured QR of the Khatri-Rao product of triangular
factors (section 3.3.3, eq. kr-id), in FP64.

Test infrastructure (see the package docstring).

The input is X = [[mu; V_1, ..., V_N]] with S terms (V_k is I_k x S, mu may
hold negative weights).  For mode n the Multi-TTM of Alg. 2 is again a
Kruskal tensor, Y = X x_{k != n} Q_k^T = [[mu; B_1, ..., B_N]] with B_n = V_n
and B_k = Q_k^T V_k (R x S) for k != n, so by eq. (cp_mat)
    Y_(n) = V_n diag(mu) (B_N (.) ... (.) B_{n+1} (.) B_{n-1} (.) ... (.) B_1)^T
and W_n = Y_(n) Q_0 = V_n diag(mu) [(... (.) B_1)^T Q_0]: Y is never formed.
For Alg. 1, M_n = X_(n) Z_n = V_n diag(mu) (Hadamard product over k != n of
V_k^T A_k), and ||X||^2 = mu^T (Hadamard product over all k of V_k^T V_k) mu.

Structured QR of V_n (the paper notes the sparsity of V_n and that its QR
need not fill in, without giving an algorithm; the reading used here): with
the modes other than n taken in increasing order a_1 < ... < a_{N-1},
T_1 = R_{a_1} and, for j = 2..N-1, the QR R_{a_j} (.) T_{j-1} = Q_j T_j of an
R^2 x R matrix (T's index fastest).  Eq. (kr-id) gives
R_{a_j} (.) (Q T) = (I_R (x) Q)(R_{a_j} (.) T), hence
    V_n = (I (x) Q_2)(I (x) Q_3) ... Q_{N-1} T_{N-1},
R_0 = T_{N-1} and Q_0 is the product of the Kronecker-structured factors.
Applied to the Kruskal columns, eq. (kr-id) again turns (... (.) B_1)^T Q_0
into a chain: C_1 = B_{a_1}, C_j = Q_j^T (B_{a_j} (.) C_{j-1}), and
(... (.) B_1)^T Q_0 = C_{N-1}^T.
"""

import numpy as np

from . import tensor as T
from . import cp_als_qr as Q
from . import cp_als as A1


def other_modes(N, n):
    """a_1 < ... < a_{N-1}: the modes other than n, increasing."""
    return [k for k in range(N) if k != n]


def krp_qr_structured(Rs, n):
    """Structured QR of V_n (reading in the module docstring).  Returns
    (Qs, R0) with Qs = [Q_2, ..., Q_{N-1}] (each R^2 x R, empty for N = 2)
    and R0 = T_{N-1}.  Library primitive: LAPACK Householder QR."""
    a = other_modes(len(Rs), n)
    Tj = np.asarray(Rs[a[0]], dtype=np.float64)
    Qs = []
    for j in range(1, len(a)):
        Qj, Tj = np.linalg.qr(T.khatri_rao(np.asarray(Rs[a[j]], dtype=np.float64), Tj), mode="reduced")
        Qs.append(Qj)
    return Qs, Tj


def q0_from_structured(Qs, R):
    """Q_0 = (I (x) Q_2)(I (x) Q_3) ... Q_{N-1} formed explicitly (R^{N-1} x R;
    the identity I_R for N = 2)."""
    if not Qs:
        return np.eye(R)
    Q0 = Qs[-1]
    for Qj in reversed(Qs[:-1]):
        m = Q0.shape[0] // R
        Q0 = np.kron(np.eye(m), Qj) @ Q0
    return Q0


def projected_factors(V, Us):
    """B_k = U_k^T V_k (R x S) for every k with U_k given (None elsewhere)."""
    return [None if U is None else np.asarray(U, dtype=np.float64).T @ np.asarray(V[k], dtype=np.float64)
            for k, U in enumerate(Us)]


def w_kruskal(mu, V, Qf, Qs, n):
    """W_n = Y_(n) Q_0 for the Kruskal input (section 3.3.2) with Q_0 in the
    structured form Qs of krp_qr_structured: the chain of eq. (kr-id) on the
    columns B_k = Q_k^T V_k, then V_n diag(mu) C_{N-1}^T."""
    N = len(V)
    a = other_modes(N, n)
    B = projected_factors(V, [None if k == n else Qf[k] for k in range(N)])
    C = B[a[0]]
    for j in range(1, len(a)):
        C = Qs[j - 1].T @ T.khatri_rao(B[a[j]], C)
    return (np.asarray(V[n], dtype=np.float64) * np.asarray(mu, dtype=np.float64)[None, :]) @ C.T


def mttkrp_kruskal(mu, V, A, n):
    """M_n = X_(n) Z_n for the Kruskal input (section 3.3.2):
    V_n diag(mu) (Hadamard product over k != n of V_k^T A_k)."""
    N = len(V)
    H = T.hadamard_list([np.asarray(V[k], dtype=np.float64).T @ np.asarray(A[k], dtype=np.float64)
                         for k in range(N) if k != n])
    return (np.asarray(V[n], dtype=np.float64) * np.asarray(mu, dtype=np.float64)[None, :]) @ H


def inner_kruskal(mu, V, lam, A):
    """<[[mu; V]], [[lam; A]]> = mu^T (Hadamard product of V_k^T A_k) lam."""
    H = T.hadamard_list([np.asarray(v, dtype=np.float64).T @ np.asarray(a, dtype=np.float64)
                         for v, a in zip(V, A)])
    return float(np.asarray(mu, dtype=np.float64) @ H @ np.asarray(lam, dtype=np.float64))


def norm2_kruskal(mu, V):
    """||X||^2 = mu^T (Hadamard product of V_k^T V_k) mu."""
    return inner_kruskal(mu, V, mu, V)


def error_gram(mu, V, lam, A, xnorm2=None):
    """||X - Xhat|| / ||X|| from Kruskal inner products (no dense tensor):
    ||X||^2 - 2 <X, Xhat> + ||Xhat||^2, resolved to about sqrt(eps) of
    the relative error by the cancellation."""
    if xnorm2 is None:
        xnorm2 = norm2_kruskal(mu, V)
    r2 = xnorm2 - 2.0 * inner_kruskal(mu, V, lam, A) + inner_kruskal(lam, A, lam, A)
    return float(np.sqrt(max(r2, 0.0)) / np.sqrt(xnorm2))


def mode_update_qr(mu, V, st, n, solver="qr", rtol=None):
    """One mode-n update of Alg. 2 for the Kruskal input: structured QR of
    V_n, W_n from the Kruskal chain, then the dense path's solve,
    normalization and factor QR.  Updates ``st`` (a cp_als_qr.State)."""
    Qs, R0 = krp_qr_structured(st.R, n)
    W = w_kruskal(mu, V, st.Q, Qs, n)
    if solver == "qr":
        Ahat, status = Q.solve_qr(W, R0)
    elif solver == "svd":
        Ahat, _, status = Q.solve_svd(W, R0, rtol)
    else:
        raise ValueError("solver must be 'qr' or 'svd'")
    A, lam = Q.normalize(Ahat)
    st.A[n], st.lam = A, lam
    st.Q[n], st.R[n] = Q.factor_qr(A)
    return dict(Qs=Qs, R0=R0, W=W, Ahat=Ahat, status=status)


def relerr(mu, V, lam, A, error, xnorm2, last=None, RN=None, Xdense=None):
    if error == "efficient":
        return Q.error_efficient(xnorm2, last["W"], last["Ahat"], last["R0"], lam, RN)
    if error == "gram":
        return error_gram(mu, V, lam, A, xnorm2)
    if error == "direct":
        X = T.full(mu, V) if Xdense is None else Xdense
        return Q.error_direct(X, lam, A)
    raise ValueError("error must be 'efficient', 'gram' or 'direct'")


def cp_als_qr_kruskal(mu, V, A_init, maxiters=25, tol=0.0, solver="qr", rtol=None, error="gram"):
    """CP-ALS-QR / CP-ALS-QR-SVD (Alg. 2) on a Kruskal input.  Returns
    (lam, A, relerr history)."""
    st = Q.init_state(A_init)
    xnorm2 = norm2_kruskal(mu, V)
    N = len(V)
    hist = []
    for s in range(maxiters):
        for n in range(N):
            last = mode_update_qr(mu, V, st, n, solver=solver, rtol=rtol)
        hist.append(relerr(mu, V, st.lam, st.A, error, xnorm2, last, st.R[N - 1]))
        if s >= 1 and abs(hist[-2] - hist[-1]) < tol:
            break
    return st.lam, st.A, hist


def cp_als_kruskal(mu, V, A_init, maxiters=25, tol=0.0, solver="chol", rtol=None, error="gram"):
    """CP-ALS / CP-ALS-PINV (Alg. 1) on a Kruskal input: the MTTKRP of
    section 3.3.2 in place of the dense one, the rest as in cp_als.  Returns
    (lam, A, relerr history)."""
    import scipy.linalg

    N = len(V)
    A = [np.array(a, dtype=np.float64) for a in A_init]
    G = [a.T @ a for a in A]
    xnorm2 = norm2_kruskal(mu, V)
    lam = np.ones(A[0].shape[1])
    hist = []
    for s in range(maxiters):
        for n in range(N):
            S = T.hadamard_list([G[k] for k in range(N) if k != n])
            M = mttkrp_kruskal(mu, V, A, n)
            if solver == "chol":
                c = scipy.linalg.cho_factor(S, lower=False, check_finite=False)
                Ahat = scipy.linalg.cho_solve(c, M.T, check_finite=False).T
            elif solver == "pinv":
                r = A1.default_rtol(S.shape[0]) if rtol is None or rtol < 0 else rtol
                Ahat = M @ np.linalg.pinv(S, rcond=r)
            else:
                raise ValueError("solver must be 'chol' or 'pinv'")
            lam = np.sqrt(np.sum(Ahat * Ahat, axis=0))
            safe = np.where(lam > 0, lam, 1.0)
            A[n] = Ahat / safe[None, :]
            G[n] = A[n].T @ A[n]
        if error == "efficient":
            ip = float(np.sum(M * Ahat))
            nn = float(np.sum(S * ((lam[:, None] * G[N - 1]) * lam[None, :])))
            rel = float(np.sqrt(max(xnorm2 - 2.0 * ip + nn, 0.0)) / np.sqrt(xnorm2))
        else:
            rel = relerr(mu, V, lam, A, error, xnorm2)
        hist.append(rel)
        if s >= 1 and abs(hist[-2] - hist[-1]) < tol:
            break
    return lam, A, hist
