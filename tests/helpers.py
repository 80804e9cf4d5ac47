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
