"""Learned initialization: a randomized sketch of the tensor, a three-layer
MLP, and a loss in Kruskal form, written out plainly in FP64.

Test infrastructure (see the package docstring).

What the GPU side computes, and what this module defines:

  sketch   X_s = X x_1 S_1 x_2 S_2 x_3 S_3 with S_k of shape (J_k, I_k)
           (TTM of section 2.2).  The MLP input is X_s flattened with the
           mode-2 index fastest, then mode 1, then mode 3:
           x[j2 + J2 j1 + J2 J1 j3] = X_s[j1, j2, j3]  (``sketch_vector``).
  MLP      h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2), y = W3 h2 + b3, with
           W_l stored (out, in).  y holds the three factor matrices one after
           the other, each column-major I x R (``unpack_factors``).
  loss     two forms, both evaluated from R x R Gram matrices
           (||[[A]]||^2 = sum of the Hadamard product of the A_k^T A_k, and
           <[[Ahat]], [[A]]> the same with Ahat_k^T A_k -- the identity that
           gives the paper's efficient error of section 3.3.1 its cheapness,
           applied to two Kruskal tensors):
             distance  ||[[Ahat]] - [[A]]||^2 / ||[[A]]||^2
             cosine    1 - <[[Ahat]], [[A]]>^2 / (||[[Ahat]]||^2 ||[[A]]||^2),
                       invariant to the scale of the prediction (CP-ALS does
                       not depend on the scale of its start).
           The loss of a batch is the mean of the per-sample losses.
  Adam     the update of Kingma and Ba with bias correction.
  HOSVD    the fallback start: for each mode k, an orthonormal basis of the
           range of X_(k) taken from its product with a Khatri-Rao test
           matrix of Gaussian factors, W_k = X_(k) (Omega_N (.) .. (.)
           Omega_{k+1} (.) Omega_{k-1} (.) .. (.) Omega_1) (the MTTKRP of
           section 2.3 with random factors), then the thin QR of W_k
           (``hosvd_start``): the randomized form of the leading-R mode-k
           singular subspace of the HOSVD (equal to it when X_(k) has rank R).

The paper does not describe this component; it is the project's learned
initializer, and the gain it brings is measured, not pinned to a published
number ("parity unpinned" for the gain).  Every function below is pinned by
tests/test_oracle_learned.py: brute-force sketch sums, the Kruskal loss
against dense reconstruction, finite-difference gradients, Adam's first step.
"""

import numpy as np

from . import tensor as T


def sketch(X, S):
    """X x_1 S[0] x_2 S[1] x_3 S[2] (each S[k] of shape J_k x I_k)."""
    Y = np.asarray(X, dtype=np.float64)
    for k, Sk in enumerate(S):
        Y = T.ttm(Y, np.asarray(Sk, dtype=np.float64), k)
    return Y


def sketch_vector(Xs):
    """Flatten a J1 x J2 x J3 sketch with j2 fastest, then j1, then j3."""
    return np.ascontiguousarray(np.transpose(Xs, (2, 0, 1))).reshape(-1)


def unpack_factors(y, I, R):
    """The output vector as three I_k x R factor matrices (column-major)."""
    out, off = [], 0
    for Ik in I:
        out.append(np.asarray(y[off:off + Ik * R], dtype=np.float64).reshape(R, Ik).T)
        off += Ik * R
    return out


def pack_factors(A):
    """Inverse of unpack_factors."""
    return np.concatenate([np.asarray(a, dtype=np.float64).T.reshape(-1) for a in A])


def relu(z):
    return np.maximum(z, 0.0)


def _keep(v):
    return v


def mlp_forward(params, x, store=_keep):
    """params = (W1, b1, W2, b2, W3, b3); x is (batch, in).  Returns y and the
    activations needed by the backward pass.  ``store`` is applied to each
    hidden activation as it is kept (identity by default; a rounding
    function models a lower-precision activation store)."""
    W1, b1, W2, b2, W3, b3 = params
    z1 = x @ W1.T + b1
    h1 = store(relu(z1))
    z2 = h1 @ W2.T + b2
    h2 = store(relu(z2))
    y = h2 @ W3.T + b3
    return y, (x, z1, h1, z2, h2)


def mlp_backward(params, cache, dy, store=_keep):
    """Gradients of a scalar loss with respect to the parameters, given dL/dy
    for every sample (chain rule through the three affine maps and ReLUs).
    ``store`` is applied to the back-propagated hidden gradients before they
    are used in the next product (identity by default)."""
    W1, b1, W2, b2, W3, b3 = params
    x, z1, h1, z2, h2 = cache
    dW3 = dy.T @ h2
    db3 = dy.sum(axis=0)
    dh2 = (dy @ W3) * (z2 > 0)
    db2 = dh2.sum(axis=0)
    dh2 = store(dh2)
    dW2 = dh2.T @ h1
    dh1 = (dh2 @ W2) * (z1 > 0)
    db1 = dh1.sum(axis=0)
    dh1 = store(dh1)
    dW1 = dh1.T @ x
    return (dW1, db1, dW2, db2, dW3, db3)


def kruskal_inner(A, B):
    """<[[A]], [[B]]> = sum over (r, s) of prod_k (A_k^T B_k)[r, s]."""
    H = np.ones((A[0].shape[1], B[0].shape[1]))
    for a, b in zip(A, B):
        H = H * (np.asarray(a, dtype=np.float64).T @ np.asarray(b, dtype=np.float64))
    return float(H.sum())


def kruskal_loss(Ahat, A):
    """||[[Ahat]] - [[A]]||^2 / ||[[A]]||^2 from Gram matrices."""
    aa = kruskal_inner(A, A)
    return (kruskal_inner(Ahat, Ahat) - 2.0 * kruskal_inner(Ahat, A) + aa) / aa


def kruskal_loss_grad(Ahat, A):
    """Loss and dL/dAhat_k for every k.

    d||[[Ahat]]||^2/dAhat_k = 2 Ahat_k G_k with G_k the Hadamard product of
    Ahat_j^T Ahat_j over j != k; d<[[Ahat]], [[A]]>/dAhat_k = A_k H_k^T with
    H_k the Hadamard product of Ahat_j^T A_j over j != k."""
    N = len(A)
    aa = kruskal_inner(A, A)
    loss = kruskal_loss(Ahat, A)
    grads = []
    for k in range(N):
        G = np.ones((Ahat[0].shape[1], Ahat[0].shape[1]))
        H = np.ones((Ahat[0].shape[1], A[0].shape[1]))
        for j in range(N):
            if j == k:
                continue
            G = G * (Ahat[j].T @ Ahat[j])
            H = H * (Ahat[j].T @ A[j])
        grads.append((2.0 * Ahat[k] @ G - 2.0 * A[k] @ H.T) / aa)
    return loss, grads


def kruskal_cosine_loss(Ahat, A):
    """1 - <[[Ahat]], [[A]]>^2 / (||[[Ahat]]||^2 ||[[A]]||^2)."""
    c = kruskal_inner(Ahat, A)
    return 1.0 - c * c / (kruskal_inner(Ahat, Ahat) * kruskal_inner(A, A))


def kruskal_cosine_loss_grad(Ahat, A):
    """Loss and gradient of the cosine form: with c = <[[Ahat]], [[A]]>,
    a = ||[[Ahat]]||^2, t = ||[[A]]||^2 and the Gram-product gradients of
    kruskal_loss_grad, dL = -(2c/(a t)) dc + (c^2/(a^2 t)) da."""
    N = len(A)
    c, a, t = kruskal_inner(Ahat, A), kruskal_inner(Ahat, Ahat), kruskal_inner(A, A)
    grads = []
    for k in range(N):
        G = np.ones((Ahat[0].shape[1], Ahat[0].shape[1]))
        H = np.ones((Ahat[0].shape[1], A[0].shape[1]))
        for j in range(N):
            if j == k:
                continue
            G = G * (Ahat[j].T @ Ahat[j])
            H = H * (Ahat[j].T @ A[j])
        dc = A[k] @ H.T
        da = 2.0 * Ahat[k] @ G
        grads.append(-(2.0 * c / (a * t)) * dc + (c * c / (a * a * t)) * da)
    return 1.0 - c * c / (a * t), grads


def batch_loss_grad(y, targets, I, R, kind="distance"):
    """Mean Kruskal loss over a batch and dL/dy (rows of y are samples;
    targets[b] is the list of target factor matrices of sample b)."""
    B = y.shape[0]
    dy = np.zeros_like(y, dtype=np.float64)
    total = 0.0
    fn = kruskal_loss_grad if kind == "distance" else kruskal_cosine_loss_grad
    for b in range(B):
        Ahat = unpack_factors(y[b], I, R)
        loss, g = fn(Ahat, targets[b])
        total += loss
        dy[b] = pack_factors(g) / B
    return total / B, dy


def adam_step(w, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba, Alg. 1) at step t >= 1; returns the new
    (w, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return w - lr * mhat / (np.sqrt(vhat) + eps), m, v


def hosvd_start(X, Omegas, R, modes=None):
    """Randomized HOSVD start: A_k = Q of the thin QR of X_(k) (Khatri-Rao of
    Omega_j, j != k) for each k in ``modes`` (default: all); the other
    entries are None.  Library primitives: the oracle's MTTKRP and LAPACK QR."""
    N = np.asarray(X).ndim
    modes = range(N) if modes is None else modes
    out = [None] * N
    for k in modes:
        W = T.mttkrp(np.asarray(X, dtype=np.float64), [np.asarray(o, dtype=np.float64) for o in Omegas], k)
        Q, _ = np.linalg.qr(W, mode="reduced")
        out[k] = Q[:, :R]
    return out
