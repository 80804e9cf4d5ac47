"""Learned-initialization kernels (bfloat16 MFMA GEMMs, sketch, Kruskal loss,
Adam) against the FP64 oracle in oracle/learned.py, on the same inputs.

Tolerances: the GPU rounds weights, inputs, activations and back-propagated
gradients to bfloat16 (relative spacing 2^-8) and accumulates in FP32.  The
oracle is run twice: with its activations and hidden gradients rounded to
bfloat16 at the points where the GPU stores them (then only the FP32
accumulation order differs: 5e-3), and in plain FP64 (2e-2 for outputs;
1e-1 for gradients, where a few ReLU masks that flip between the two
roundings move whole rows).  The Kruskal loss kernel reads FP32 values and
sums in FP64 (1e-4); Adam is elementwise FP32 (1e-5)."""

import numpy as np
import pytest
import torch

from oracle import learned as OL
from oracle.precision import round_bf16
from paper_2112_10855_amd import cpqr as C
from helpers import relnorm, to_dev, to_np

pytestmark = pytest.mark.gpu


def bf16_dev(a):
    """Host array -> device FP32 -> bfloat16 through the library."""
    return C.cpqr_to_bf16(torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda"))


def up(t):
    return t.float().cpu().numpy().astype(np.float64)


def rbf(a):
    """Round to bfloat16 (the oracle's bit-level rounding), as FP64."""
    return round_bf16(np.asarray(a, dtype=np.float32)).astype(np.float64)


def make_net(rng, din, hid, dout):
    Ws = [rng.standard_normal((hid, din)) / np.sqrt(din), rng.standard_normal((hid, hid)) / np.sqrt(hid),
          rng.standard_normal((dout, hid)) / np.sqrt(hid)]
    bs = [rng.standard_normal(hid) * 0.1, rng.standard_normal(hid) * 0.1, rng.standard_normal(dout) * 0.1]
    Wb = [bf16_dev(w) for w in Ws]
    bd = [torch.as_tensor(b, dtype=torch.float32, device="cuda") for b in bs]
    # oracle parameters: the bfloat16 weights as the GPU holds them, FP32 biases
    params = [up(Wb[0]), bd[0].cpu().numpy().astype(np.float64), up(Wb[1]), bd[1].cpu().numpy().astype(np.float64),
              up(Wb[2]), bd[2].cpu().numpy().astype(np.float64)]
    return C.MlpNet(Wb, bd), params


@pytest.mark.parametrize("din,hid,dout,batch", [(128, 64, 192, 64), (256, 128, 384, 128)])
def test_mlp_forward_matches_oracle(din, hid, dout, batch):
    rng = np.random.default_rng(din + hid)
    net, params = make_net(rng, din, hid, dout)
    xb = bf16_dev(rng.standard_normal((batch, din)))
    y, (_, h1, _) = net.forward(xb)
    torch.cuda.synchronize()
    yr, cr = OL.mlp_forward(params, up(xb), store=rbf)
    assert relnorm(y.cpu().numpy(), yr) < 5e-3
    assert relnorm(up(h1), cr[2]) < 5e-3
    yo, cache = OL.mlp_forward(params, up(xb))
    assert relnorm(y.cpu().numpy(), yo) < 2e-2
    assert relnorm(up(h1), cache[2]) < 2e-2


def test_mlp_backward_matches_oracle():
    rng = np.random.default_rng(11)
    din, hid, dout, batch = 256, 64, 192, 64
    net, params = make_net(rng, din, hid, dout)
    xb = bf16_dev(rng.standard_normal((batch, din)))
    y, cache = net.forward(xb)
    dyb = bf16_dev(rng.standard_normal((batch, dout)) / batch)
    dy = dyb.float().contiguous()
    dW = [torch.empty(hid, din, device="cuda"), torch.empty(hid, hid, device="cuda"), torch.empty(dout, hid, device="cuda")]
    db = [torch.empty(hid, device="cuda"), torch.empty(hid, device="cuda"), torch.empty(dout, device="cuda")]
    net.backward(cache, dy, dyb, dW, db)
    torch.cuda.synchronize()
    _, rcache = OL.mlp_forward(params, up(xb), store=rbf)
    gr = OL.mlp_backward(params, rcache, up(dyb), store=rbf)
    _, ocache = OL.mlp_forward(params, up(xb))
    g = OL.mlp_backward(params, ocache, up(dyb))
    for l in range(3):
        assert relnorm(dW[l].cpu().numpy(), gr[2 * l]) < 5e-3, l
        assert relnorm(db[l].cpu().numpy(), gr[2 * l + 1]) < 5e-3, l
        assert relnorm(dW[l].cpu().numpy(), g[2 * l]) < 1e-1, l
        assert relnorm(db[l].cpu().numpy(), g[2 * l + 1]) < 1e-1, l


@pytest.mark.parametrize("kind", ["distance", "cosine"])
@pytest.mark.parametrize("I,R,Rt", [((32, 40, 24), 3, 3), ((256, 256, 256), 10, 10), ((17, 5, 9), 2, 4)])
def test_kruskal_loss_grad_matches_oracle(I, R, Rt, kind):
    rng = np.random.default_rng(sum(I) + R)
    B = 5
    y = rng.standard_normal((B, sum(I) * R)).astype(np.float32)
    t = rng.standard_normal((B, sum(I) * Rt)).astype(np.float32)
    code = C.LOSS_DISTANCE if kind == "distance" else C.LOSS_COSINE
    loss, dy, dyb = C.cpqr_kruskal_loss_grad(torch.as_tensor(y, device="cuda"), torch.as_tensor(t, device="cuda"),
                                             I, R, Rt, scale=1.0 / B, kind=code)
    torch.cuda.synchronize()
    targets = [OL.unpack_factors(t[b].astype(np.float64), I, Rt) for b in range(B)]
    lo, dyo = OL.batch_loss_grad(y.astype(np.float64), targets, I, R, kind=kind)
    one = OL.kruskal_loss if kind == "distance" else OL.kruskal_cosine_loss
    assert abs(float(loss.mean()) - lo) < 1e-4 * max(1.0, abs(lo))
    for b in range(B):
        ob = one(OL.unpack_factors(y[b].astype(np.float64), I, R), targets[b])
        assert abs(float(loss[b]) - ob) < 1e-4 * max(1.0, abs(ob))
    assert relnorm(dy.cpu().numpy(), dyo) < 1e-4
    assert relnorm(up(dyb), dyo) < 1e-2


@pytest.mark.parametrize("shape", [(64, 64, 64), (96, 64, 128)])
def test_sketch_matches_oracle(shape):
    rng = np.random.default_rng(sum(shape))
    X = rng.standard_normal(shape).astype(np.float32)
    S = [rng.standard_normal((64, n)) / 8.0 for n in shape]
    Sb = [bf16_dev(s) for s in S]
    Xd = C.colmajor(torch.as_tensor(X, device="cuda"))
    xs, xb = C.cpqr_sketch3(Xd, Sb)
    torch.cuda.synchronize()
    ref = OL.sketch_vector(OL.sketch(X.astype(np.float64), [up(s) for s in Sb]))
    assert relnorm(xs.cpu().numpy(), ref) < 2e-2
    xn = up(xb)
    assert abs(np.linalg.norm(xn) / np.sqrt(xn.size) - 1.0) < 1e-2  # unit RMS
    assert relnorm(xn, ref * np.sqrt(ref.size) / np.linalg.norm(ref)) < 2e-2


def test_adam_matches_oracle():
    rng = np.random.default_rng(12)
    n = 10000
    w = rng.standard_normal(n).astype(np.float32)
    m = (rng.standard_normal(n) * 0.01).astype(np.float32)
    v = (rng.random(n) * 0.01).astype(np.float32)
    g = rng.standard_normal(n).astype(np.float32)
    wd, md, vd, gd = [torch.as_tensor(a, device="cuda") for a in (w, m, v, g)]
    wb = torch.empty(n, dtype=torch.bfloat16, device="cuda")
    C.cpqr_adam(wd, gd, md, vd, wb, step=3, lr=1e-3)
    torch.cuda.synchronize()
    wo, mo, vo = OL.adam_step(w.astype(np.float64), g.astype(np.float64), m.astype(np.float64),
                              v.astype(np.float64), 3, 1e-3)
    assert relnorm(wd.cpu().numpy(), wo) < 1e-5
    assert relnorm(md.cpu().numpy(), mo) < 1e-5
    assert relnorm(vd.cpu().numpy(), vo) < 1e-5
    assert relnorm(up(wb), wo) < 1e-2


def test_training_steps_reduce_the_loss():
    """Adam steps of the GPU forward/backward on one batch lower the cosine
    Kruskal loss steadily (the gradient points downhill)."""
    rng = np.random.default_rng(13)
    I, R = (32, 32, 32), 2
    din, hid, dout, batch = 128, 64, 3 * 32 * 2, 64
    Ws = [rng.standard_normal((hid, din)) / np.sqrt(din), rng.standard_normal((hid, hid)) / np.sqrt(hid),
          rng.standard_normal((dout, hid)) / np.sqrt(hid)]
    W = [torch.as_tensor(w, dtype=torch.float32, device="cuda").contiguous() for w in Ws]
    b = [torch.zeros(hid, device="cuda"), torch.zeros(hid, device="cuda"), torch.zeros(dout, device="cuda")]
    Wb = [C.cpqr_to_bf16(w) for w in W]
    net = C.MlpNet(Wb, b)
    params = W + b
    mom = [torch.zeros_like(p) for p in params]
    vel = [torch.zeros_like(p) for p in params]
    xb = bf16_dev(rng.standard_normal((batch, din)))
    tgt = torch.as_tensor(rng.standard_normal((batch, dout)) * 0.3, dtype=torch.float32, device="cuda")
    dW = [torch.empty_like(w) for w in W]
    db = [torch.empty_like(x) for x in b]
    losses = []
    for step in range(1, 31):
        y, cache = net.forward(xb)
        loss, dy, dyb = C.cpqr_kruskal_loss_grad(y, tgt, I, R, R, scale=1.0 / batch, kind=C.LOSS_COSINE)
        losses.append(float(loss.mean()))
        net.backward(cache, dy, dyb, dW, db)
        for k, (p, gr) in enumerate(zip(params, dW + db)):
            C.cpqr_adam(p, gr, mom[k], vel[k], Wb[k] if k < 3 else None, step, 3e-3)
    torch.cuda.synchronize()
    assert losses[-1] < 0.95 * losses[0], losses
    assert all(b <= a + 1e-3 for a, b in zip(losses, losses[1:])), losses


@pytest.mark.parametrize("shape,R,prec", [((30, 25, 20), 4, "f64"), ((64, 50, 40), 10, "f64"), ((64, 50, 40), 10, "f32"),
                                          ((9, 8, 10, 7), 3, "f64")])
def test_hosvd_init_against_oracle(shape, R, prec):
    """The randomized HOSVD start (cpqr_hosvd_init) against the oracle with
    the same Gaussian test factors: the QR of X_(k) (Khatri-Rao of Omega_j)
    is unique up to column signs, so the bases are compared after fixing
    them, entry by entry (FP64 Multi-TTM: 1e-10; FP32: 1e-4, the FP32
    Multi-TTM error amplified by cond(W_k)).  For an exact rank-R tensor the
    basis also spans the ground-truth factor."""
    import oracle.learned as OLm
    from oracle import tensor as OT
    g = np.random.default_rng(sum(shape) + R)
    A = [g.standard_normal((s, R)) for s in shape]
    X = OT.full(np.ones(R), A) + 1e-3 * g.standard_normal(shape)
    Om = [g.standard_normal((s, R)) for s in shape]
    tdt = torch.float64 if prec == "f64" else torch.float32
    Q = C.cpqr_hosvd_init(to_dev(X.astype(np.float32) if prec == "f32" else X, tdt), [to_dev(o) for o in Om], R,
                          prec=C.PREC_F64 if prec == "f64" else C.PREC_F32, k0=1)
    Xo = X.astype(np.float32).astype(np.float64) if prec == "f32" else X
    ref = OLm.hosvd_start(Xo, Om, R)
    tol = 1e-10 if prec == "f64" else 1e-4
    assert Q[0] is None
    for k in range(1, len(shape)):
        q = to_np(Q[k])
        d = np.sign(np.sum(q * ref[k], axis=0))
        np.testing.assert_allclose(q * d[None, :], ref[k], rtol=0, atol=tol)
        np.testing.assert_allclose(q.T @ q, np.eye(R), rtol=0, atol=1e-12)
