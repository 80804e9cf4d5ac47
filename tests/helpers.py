"""Shared test plumbing: moving seeded numpy inputs to the GPU in the
library's column-major layout and back.  No arithmetic of the method."""

import numpy as np
import torch

from paper_2112_10855_amd import cpqr as C


def to_dev(a, dtype=torch.float64):
    """numpy array -> column-major CUDA tensor with the same values."""
    a = np.asarray(a)
    flat = torch.from_numpy(np.ascontiguousarray(a.ravel(order="F")))
    t = flat.to(device="cuda", dtype=dtype)
    rev = list(reversed(a.shape))
    perm = list(reversed(range(a.ndim)))
    return t.view(rev).permute(perm)


def to_np(t):
    return t.detach().cpu().numpy()


def sign_fix(Q, R):
    """Flip signs so that diag(R) >= 0 (Q R unchanged)."""
    d = np.sign(np.diag(R))
    d[d == 0] = 1.0
    return Q * d[None, :], d[:, None] * R


def relnorm(a, b):
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(np.asarray(a, dtype=np.float64) - b) / max(np.linalg.norm(b), 1e-300))


def abs_bound_multittm(X, Qs, n):
    """|X| x_{k != n} |Q_k|^T unfolded along n: entry by entry, the sum of the
    magnitudes of the products that make up that entry of Y_(n).  Every
    rounding error of a Multi-TTM is a multiple of these products, so
    per-entry tolerances are stated relative to this bound."""
    import oracle.cp_als_qr as OQ
    return OQ.multittm_unfolded(np.abs(np.asarray(X, dtype=np.float64)),
                                [None if q is None else np.abs(np.asarray(q, dtype=np.float64)) for q in Qs], n)


def assert_entrywise(Y, Yo, bound, tol, ctx=""):
    """|Y - Yo| <= tol * bound for every entry (NaN fails).  Returns the
    largest ratio |Y - Yo| / (tol * bound) for reporting."""
    Y = np.asarray(Y, dtype=np.float64)
    Yo = np.asarray(Yo, dtype=np.float64)
    bound = np.asarray(bound, dtype=np.float64)
    assert Y.shape == Yo.shape, (ctx, Y.shape, Yo.shape)
    err = np.abs(Y - Yo)
    lim = tol * bound
    ok = err <= lim
    ratio = np.where(lim > 0, err / np.where(lim > 0, lim, 1.0), np.where(err > 0, np.inf, 0.0))
    if not ok.all():
        bad = np.argwhere(~ok)
        i = tuple(bad[np.argmax(ratio[~ok])]) if np.isfinite(ratio[~ok]).any() else tuple(bad[0])
        raise AssertionError("%s: %d of %d entries off; worst at %s: got %r want %r bound %r tol %g"
                             % (ctx, len(bad), err.size, i, Y[i], Yo[i], bound[i], tol))
    return float(ratio.max()) if ratio.size else 0.0


def multittm_tol_f32(shape, n):
    """Per-entry tolerance of the FP32 Multi-TTM relative to the magnitude
    bound: 1e-5, the FP32 contract.  (A bad entry -- a wrong index, a lost
    tile -- is off by about |Y|, 1/sqrt(K) of the bound or more.)"""
    return 1e-5


def multittm_tol_lowp(shape, n, mode):
    """Per-entry tolerance of the reduced-precision forms relative to the
    magnitude bound, per contraction: split bfloat16 keeps each product to
    3 * 2^-18 (the dropped x_lo q_lo and the two split residuals) and plain
    bfloat16 to 2^-8 (both operands rounded); the FP32 accumulation and the
    FP32 intermediates add K * 2^-24 at worst.  One such term per contraction."""
    steps = len(shape) - 1
    kmax = max(s for k, s in enumerate(shape) if k != n)
    per = (3.1 * 2.0 ** -16 if mode == "bf16x2" else 2.1 * 2.0 ** -9) + (kmax + 2) * 2.0 ** -24
    return steps * per


def kruskal_distance(l1, A1, l2, A2):
    """||[[l1; A1]] - [[l2; A2]]|| / ||[[l2; A2]]|| through Gram matrices:
    <[[a]], [[b]]> = a^T (Hadamard product of A_k^T B_k) b.  The squared
    distance is a difference of terms of size ||[[l2; A2]]||^2, so distances
    below about 1e-8 (the square root of the FP64 spacing) are not resolved;
    compare dense models or the factors themselves below that."""
    def ip(la, A, lb, B):
        H = np.ones((len(la), len(lb)))
        for a, b in zip(A, B):
            H = H * (a.T @ b)
        return float(la @ H @ lb)
    d2 = ip(l1, A1, l1, A1) - 2 * ip(l1, A1, l2, A2) + ip(l2, A2, l2, A2)
    return float(np.sqrt(max(d2, 0.0) / ip(l2, A2, l2, A2)))
