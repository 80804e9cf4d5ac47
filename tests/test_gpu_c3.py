"""Parity at the 4-way precision-study workload: a 200 x 200 x 200 x 200
FP32 tensor (6.4 GB) with a rank-32 ground truth whose weights spread over
1e0..1e-6, no noise, through the same C-ABI calls the benchmark times.

  * Multi-TTM for every mode in FP32, split bfloat16 and plain bfloat16
    (eq. multittm): sampled rows of Y_(n), each computed by the oracle from
    the single slab X(.., i_n, ..) it depends on, checked entry by entry
    against the per-contraction error bound of each form.  At R = 32 the
    first contraction runs the row-tiled matrix-core kernels with two
    16-column blocks and wide row tiles (4 x 64 rows per wavefront in FP32,
    2 x 64 in bfloat16): with non-temporal tensor loads when the contracted
    mode's rows are 40000 elements apart (mode 2) and without when they are
    200 apart (modes 1, 3, 4).
  * One CP-ALS-QR sweep (Alg. 2, with the mode reuse the benchmark uses)
    from the shared start against one oracle sweep on the same bytes.
"""

import functools

import numpy as np
import pytest
import torch

import oracle.cp_als_qr as OQ
from paper_2112_10855_amd import cpqr as C
from paper_2112_10855_amd import synth
from helpers import (abs_bound_multittm, assert_entrywise, kruskal_distance, multittm_tol_f32, multittm_tol_lowp,
                     relnorm, to_np)

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

N1 = 200
R = 32
ROWS = (0, 1, 63, 64, 127, 128, N1 - 1)


@pytest.fixture(scope="module")
def c3():
    print("\n[c3] generating %d^4 FP32 workload, rank %d" % (N1, R), flush=True)
    d = synth.workload_4way(n=N1, R=R)
    X = d["X"]
    Xd = torch.from_numpy(X.reshape(-1, order="F")).to("cuda").view(N1, N1, N1, N1).permute(3, 2, 1, 0)
    torch.cuda.synchronize()
    Qs = [synth.orthonormal_columns(N1, R, 70 + k) for k in range(4)]

    @functools.lru_cache(maxsize=None)
    def slab_ref(n, i):
        sl = [slice(None)] * 4
        sl[n] = slice(i, i + 1)
        sub = X[tuple(sl)].astype(np.float64)
        return OQ.multittm_unfolded(sub, Qs, n)[0], abs_bound_multittm(sub, Qs, n)[0]

    return d, Xd, Qs, slab_ref


@pytest.mark.parametrize("prec", ["f32", "bf16x2", "bf16"])
def test_c3_multittm_sampled_rows(c3, prec):
    d, Xd, Qs, slab_ref = c3
    Qd = [torch.from_numpy(q).to("cuda").t().contiguous().t() for q in Qs]
    shape = d["X"].shape
    for n in range(4):
        print("[c3] multittm %s mode %d" % (prec, n), flush=True)
        Y = to_np(C.cpqr_multittm(Xd, [None if k == n else Qd[k] for k in range(4)], n, prec))
        tol = multittm_tol_f32(shape, n) if prec == "f32" else multittm_tol_lowp(shape, n, prec)
        errs = []
        for i in ROWS:
            yo, bound = slab_ref(n, i)
            assert_entrywise(Y[i], yo, bound, tol, (prec, n, i))
            errs.append(relnorm(Y[i], yo))
        print("[c3] %s mode %d: relative error of the sampled rows %.2e" % (prec, n, max(errs)), flush=True)


def test_c3_one_sweep_against_oracle(c3):
    d, Xd, _, _ = c3
    st = C.AlsState(Xd, d["init"], prec=C.PREC_F32)
    st.init()
    rel = st.sweep(1).cpu().numpy()
    lam = to_np(st.lam)
    A = [to_np(a) for a in st.A]
    print("[c3] oracle sweep", flush=True)
    X64 = d["X"].astype(np.float64)
    ost = OQ.init_state(d["init"])
    orel, _ = OQ.sweep(X64, ost)
    del X64
    dist = kruskal_distance(lam, A, ost.lam, ost.A)
    fac = [relnorm(A[k], ost.A[k]) for k in range(4)]
    print("[c3] sweep: relerr gpu %.8e oracle %.8e; model distance %.2e; factors %s"
          % (rel[0], orel, dist, ["%.2e" % f for f in fac]), flush=True)
    assert abs(rel[0] ** 2 - orel ** 2) < 2e-6
    assert dist < 1e-4
