"""Seeded synthetic inputs shaped like the paper's workloads.

This module is shared by the tests, the benchmark and the smoke check; it
holds none of CP-ALS-QR's arithmetic.  It only draws random numbers and
builds data tensors of known CP structure:

  X = sum_r lam_r a_r^(1) o ... o a_r^(N)  +  noise                (eq. cp)

with the recipes of the paper's experiments (section 4): Gaussian factor
entries, factors with controlled collinearity (section 4.2, collinearity
through Cholesky mixing of orthonormal columns), relative Gaussian noise,
and random initial factors shared by every method.

Tensors are returned as Fortran-ordered numpy arrays of shape
(I_1, ..., I_N): mode 1 is the fastest-varying index in memory, which is the
layout the GPU library expects.  All randomness is numpy PCG64 seeded through
SeedSequence, so a seed fixes every byte independently of thread count.
"""

import concurrent.futures as _cf
import os

import numpy as np

_SUBSCRIPTS = "abcdefghij"


def _children(seed, n):
    return np.random.SeedSequence(int(seed)).spawn(n)


def _gen(ss):
    return np.random.Generator(np.random.PCG64(ss))


def gaussian_factors(shape, R, seed):
    """Factor matrices with iid N(0,1) entries, one I_k x R array per mode."""
    kids = _children(seed, len(shape))
    return [_gen(kids[k]).standard_normal((int(shape[k]), R)) for k in range(len(shape))]


def init_factors(shape, R, seed):
    """Random initial factors (iid N(0,1)), shared by every method under test
    (section 4.2 and 4.3 give all methods the same random start)."""
    return gaussian_factors(shape, R, seed + 7919)


def orthonormal_columns(I, R, seed):
    """An I x R matrix with orthonormal columns (orthonormalized Gaussian)."""
    G = _gen(np.random.SeedSequence(int(seed))).standard_normal((int(I), R))
    Q, _ = np.linalg.qr(G)
    return Q


def collinear_factors(shape, R, congruence, seed):
    """Factors with unit columns and pairwise column cosine ``congruence``:
    A_k = orth(Gaussian) U with U^T U = (1-c) I + c 11^T (Cholesky mixing)."""
    c = float(congruence)
    Gm = (1.0 - c) * np.eye(R) + c * np.ones((R, R))
    U = np.linalg.cholesky(Gm).T
    kids = _children(seed, len(shape))
    out = []
    for k in range(len(shape)):
        G = _gen(kids[k]).standard_normal((int(shape[k]), R))
        Qk, _ = np.linalg.qr(G)
        out.append(Qk @ U)
    return out


def log_spread_weights(R, decades):
    """lam_r = 10^(-decades (r-1)/(R-1)), r = 1..R."""
    if R == 1:
        return np.ones(1)
    return 10.0 ** (-decades * np.arange(R) / (R - 1))


def _slab(lam, A, lo, hi):
    """Noise-free model restricted to last-mode indices [lo, hi), float64."""
    N = len(A)
    subs = ",".join(_SUBSCRIPTS[k] + "z" for k in range(N))
    out = _SUBSCRIPTS[:N]
    ops = [A[k] * (lam[None, :] if k == 0 else 1.0) for k in range(N - 1)] + [A[N - 1][lo:hi]]
    return np.einsum(subs + "->" + out, *ops, optimize=True)


def _chunks(last, per):
    return [(lo, min(lo + per, last)) for lo in range(0, last, per)]


def cp_tensor(shape, R, seed, *, weights=None, factors=None, congruence=None,
              normalize_columns=False, noise=0.0, dtype=np.float32, threads=None):
    """A dense tensor with exact rank-R CP structure plus relative noise.

    Returns dict(X, lam, A).  ``noise`` is eta: X = X0 + eta ||X0|| E / sqrt(|X|)
    with E iid N(0,1), so the noise has norm about eta ||X0||.  X is built
    slab by slab along the last mode in float64 and stored in ``dtype``.
    """
    shape = tuple(int(s) for s in shape)
    N = len(shape)
    if factors is not None:
        A = [np.array(a, dtype=np.float64) for a in factors]
    elif congruence is not None:
        A = collinear_factors(shape, R, congruence, seed)
    else:
        A = gaussian_factors(shape, R, seed)
    if normalize_columns:
        A = [a / np.sqrt(np.sum(a * a, axis=0))[None, :] for a in A]
    lam = np.ones(R) if weights is None else np.asarray(weights, dtype=np.float64)

    size = int(np.prod(shape))
    slab_elems = size // shape[-1]
    per = max(1, min(shape[-1], (1 << 24) // max(1, slab_elems)))
    chunks = _chunks(shape[-1], per)
    noise_kids = _children(seed + 104729, len(chunks))
    nthreads = threads or min(16, os.cpu_count() or 1)

    X = np.empty(shape, dtype=dtype, order="F")
    flat = X.reshape(-1, order="F")

    def norm2_of(ci):
        lo, hi = chunks[ci]
        s = _slab(lam, A, lo, hi)
        return float(np.sum(s * s))

    scale = 0.0
    if noise > 0.0:
        with _cf.ThreadPoolExecutor(nthreads) as ex:
            x0norm2 = sum(ex.map(norm2_of, range(len(chunks))))
        scale = float(noise) * np.sqrt(x0norm2) / np.sqrt(size)

    def fill(ci):
        lo, hi = chunks[ci]
        s = _slab(lam, A, lo, hi).reshape(-1, order="F")
        if scale > 0.0:
            e = _gen(noise_kids[ci]).standard_normal(s.size)
            s = s + scale * e
        flat[lo * slab_elems: hi * slab_elems] = s.astype(dtype)

    with _cf.ThreadPoolExecutor(nthreads) as ex:
        list(ex.map(fill, range(len(chunks))))
    return dict(X=X, lam=lam, A=A)


# The paper-shaped workloads.  Seeds follow data = 1000*c + b, init = 2000*c + b
# for workload c and item b.

def workload_small(noise=1e-4, seed_item=1):
    """50x50x50 FP64, rank-5 Gaussian ground truth, relative noise 1e-4
    (section 4.2 tensor size and rank); CP-ALS-QR rank 5 from a seeded start."""
    d = cp_tensor((50, 50, 50), 5, 1000 + seed_item, noise=noise, dtype=np.float64)
    d["init"] = init_factors((50, 50, 50), 5, 2000 + seed_item)
    d["R"] = 5
    return d


def workload_large3(n=1000, R=16, congruence=0.99, noise=1e-3, seed_item=0, threads=None):
    """n^3 FP32 (4 GB at n=1000), rank-16 ground truth with column congruence
    0.99 (Cholesky mixing), relative noise 1e-3."""
    shape = (n, n, n)
    d = cp_tensor(shape, R, 2000 + seed_item, congruence=congruence, noise=noise,
                  dtype=np.float32, threads=threads)
    d["init"] = init_factors(shape, R, 4000 + seed_item)
    d["R"] = R
    return d


def workload_4way(n=200, R=32, seed_item=0, threads=None):
    """n^4 FP32, rank-32 ground truth with unit Gaussian columns and weights
    spread over 1e0..1e-6, no noise."""
    shape = (n, n, n, n)
    d = cp_tensor(shape, R, 3000 + seed_item, weights=log_spread_weights(R, 6.0),
                  normalize_columns=True, dtype=np.float32, threads=threads)
    d["init"] = init_factors(shape, R, 6000 + seed_item)
    d["R"] = R
    return d


def batch_shapes(count=512, lo=20, hi=160, rlo=2, rhi=12, seed=4000):
    """Uneven 3-way shapes and ranks for a batch of independent tensors:
    each mode size uniform in [lo, hi], rank uniform in [rlo, rhi]."""
    g = _gen(np.random.SeedSequence(seed))
    dims = g.integers(lo, hi + 1, size=(count, 3))
    ranks = g.integers(rlo, rhi + 1, size=count)
    return [(tuple(int(v) for v in dims[b]), int(ranks[b])) for b in range(count)]


# ---------------------------------------------------------------- sine of sums
# The function-approximation workload of section 4.3: sin(x_1 + ... + x_N)
# on an n-point grid of [0, 2 pi) per variable, a tensor of exact CP rank at
# most N with a known rank-2^{N-1} expansion.

def sine_of_sums_grid(n):
    """x_j: n points discretizing [0, 2 pi) (x_i = 2 pi i / n, i = 0..n-1)."""
    return 2.0 * np.pi * np.arange(int(n), dtype=np.float64) / int(n)


def sine_of_sums(N, n, dtype=np.float64):
    """Dense X[i_1, ..., i_N] = sin(x_{i_1} + ... + x_{i_N}), Fortran order;
    the sums and sines are taken in FP64, then cast to ``dtype``."""
    x = sine_of_sums_grid(n)
    S = np.zeros((int(n),) * N, dtype=np.float64, order="F")
    for k in range(N):
        sh = [1] * N
        sh[k] = int(n)
        S += x.reshape(sh)
    np.sin(S, out=S)
    return S if dtype == np.float64 else np.asfortranarray(S.astype(dtype))


def sine_of_sums_expanded(N, n):
    """The rank-2^{N-1} CP form from the sum identities of sine and cosine:
    one term per set J of variables of odd size, sign (-1)^{(|J|-1)/2},
    factor sin(x) in the modes of J and cos(x) elsewhere.  Returns (lam, A)."""
    x = sine_of_sums_grid(n)
    s, c = np.sin(x), np.cos(x)
    cols = [[] for _ in range(N)]
    lam = []
    for mask in range(1 << N):
        k = bin(mask).count("1")
        if k % 2 == 0:
            continue
        lam.append(-1.0 if (k - 1) // 2 % 2 else 1.0)
        for j in range(N):
            cols[j].append(s if mask >> j & 1 else c)
    return np.array(lam), [np.stack(cj, axis=1) for cj in cols]


def sine_of_sums_rank_n(N, n, alpha):
    """The rank-N CP form of eq. (sinsum_rkd): term j has sin(x) in mode j
    and sin(x + alpha_k - alpha_j) / sin(alpha_k - alpha_j) in every other
    mode k (the alpha_j pairwise distinct modulo pi).  Returns (lam, A)."""
    x = sine_of_sums_grid(n)
    alpha = np.asarray(alpha, dtype=np.float64)
    A = []
    for k in range(N):
        M = np.empty((int(n), N))
        for j in range(N):
            M[:, j] = np.sin(x) if k == j else np.sin(x + alpha[k] - alpha[j]) / np.sin(alpha[k] - alpha[j])
        A.append(M)
    return np.ones(N), A
