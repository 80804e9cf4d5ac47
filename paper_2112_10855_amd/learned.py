"""Learned initialization for CP-ALS-QR on 3-way tensors.

A fixed Gaussian sketch of the tensor (X x_1 S_1 x_2 S_2 x_3 S_3, S_k of
size J x I_k with entries N(0, 1/J)), scaled to unit root-mean-square, feeds a
three-layer MLP (ReLU, width ``hidden``, bfloat16 weights with FP32 master
copies and Adam) whose output holds the three initial factor matrices.  The
network is trained on tensors whose targets are the factors the batched
GPU CP-ALS-QR itself reached, with the scale-free Kruskal-form loss
1 - <[[Ahat]], [[A*]]>^2 / (||[[Ahat]]||^2 ||[[A*]]||^2) (CP-ALS does not depend
on the scale of its start; the distance form has a flat saddle at zero and
grows with the sixth power of the output).
At inference only A_2 and A_3 of the prediction are used (Alg. 2 never
reads the initial A_1); the fallback is the randomized HOSVD start
(cpqr_hosvd_init: an orthonormal basis of the range of X_(k) sampled by a
Khatri-Rao test matrix of Gaussian factors).

Every step runs in libcpqr's kernels (sketch, GEMMs, loss gradient, Adam,
batched CP-ALS-QR); torch provides device memory and builds the synthetic
input tensors from their factors.
"""

import time

import numpy as np
import torch

from . import cpqr as C
from . import synth


def c5_factors(shape, R, seed, congruence=0.9):
    """Ground-truth factors of the learned-init workload: unit columns with
    pairwise cosine ``congruence`` (Cholesky mixing), weights 1."""
    return synth.collinear_factors(shape, R, congruence, seed)


def build_tensor(A, device="cuda"):
    """Dense column-major FP32 tensor [[A_1, A_2, A_3]] on the device (input
    construction: X_(1) = A_1 (A_3 (.) A_2)^T)."""
    A = [torch.as_tensor(a, dtype=torch.float32, device=device) for a in A]
    I1, I2, I3 = (a.shape[0] for a in A)
    R = A[0].shape[1]
    kr = (A[2][:, None, :] * A[1][None, :, :]).reshape(I3 * I2, R)  # row i2 + I2 i3
    Xt = kr @ A[0].T  # (I2 I3) x I1, row-major == column-major X
    return Xt.contiguous().view(I3, I2, I1).permute(2, 1, 0)


class LearnedInit:
    def __init__(self, shape=(256, 256, 256), R=10, J=64, hidden=512, seed=0, device="cuda"):
        self.shape, self.R, self.J, self.hidden = tuple(int(s) for s in shape), int(R), int(J), int(hidden)
        self.device = device
        rng = np.random.default_rng(seed)
        S = [rng.standard_normal((J, n)) / np.sqrt(J) for n in self.shape]
        self.S = [C.cpqr_to_bf16(torch.as_tensor(s, dtype=torch.float32, device=device).contiguous()) for s in S]
        self.din = J ** 3
        self.dout = sum(self.shape) * self.R
        dims = [(hidden, self.din), (hidden, hidden), (self.dout, hidden)]
        self.W = [torch.as_tensor(rng.standard_normal(d) * np.sqrt(2.0 / d[1]), dtype=torch.float32,
                                  device=device).contiguous() for d in dims]
        # output head small enough that the first predicted Kruskal tensors
        # have norm of order one (the loss has a flat saddle at zero output)
        self.W[2].mul_(0.04)
        self.b = [torch.zeros(d[0], dtype=torch.float32, device=device) for d in dims]
        self.Wb = [C.cpqr_to_bf16(w) for w in self.W]
        self.net = C.MlpNet(self.Wb, self.b)
        self.params = self.W + self.b
        self.m = [torch.zeros_like(p) for p in self.params]
        self.v = [torch.zeros_like(p) for p in self.params]
        self.dW = [torch.empty_like(w) for w in self.W]
        self.db = [torch.empty_like(x) for x in self.b]
        self.step = 0

    def sketch(self, X):
        """Unit-RMS bfloat16 sketch vector of a column-major FP32 tensor."""
        return C.cpqr_sketch3(X, self.S)[1]

    def forward(self, xb):
        return self.net.forward(xb)

    def train_step(self, xb, targets, lr):
        """One Adam step on a batch (rows of xb: sketches; rows of targets:
        packed target factors).  Returns the per-sample losses (device)."""
        y, cache = self.net.forward(xb)
        B = xb.shape[0]
        loss, dy, dyb = C.cpqr_kruskal_loss_grad(y, targets, self.shape, self.R, self.R, scale=1.0 / B,
                                                 kind=C.LOSS_COSINE)
        self.net.backward(cache, dy, dyb, self.dW, self.db)
        self.step += 1
        for k, (p, g) in enumerate(zip(self.params, self.dW + self.db)):
            C.cpqr_adam(p, g, self.m[k], self.v[k], self.Wb[k] if k < 3 else None, self.step, lr)
        return loss

    def predict(self, xb):
        """Predicted factor matrices for a batch of sketches: list over
        samples of [A_1, A_2, A_3] (FP64 host arrays)."""
        y, _ = self.net.forward(xb)
        y = y.double().cpu().numpy()
        out = []
        for row in y:
            fac, off = [], 0
            for n in self.shape:
                fac.append(row[off:off + n * self.R].reshape(self.R, n).T.copy())
                off += n * self.R
            out.append(fac)
        return out


def pack_targets(A, lam):
    """Target row: [A_1 diag(lam) / ||[[lam; A]]||, A_2, A_3], column-major,
    FP32 (the Kruskal norm from R x R Gram matrices)."""
    H = np.outer(lam, lam)
    for a in A:
        H = H * (a.T @ a)
    nrm = np.sqrt(max(H.sum(), 1e-300))
    A1 = A[0] * (lam[None, :] / nrm)
    return np.concatenate([A1.T.reshape(-1), A[1].T.reshape(-1), A[2].T.reshape(-1)]).astype(np.float32)


def make_dataset(model, count, seed0, sweeps=100, chunk=256, log=print):
    """Sketches (bfloat16, count x J^3) and method targets (FP32, count x dout)
    for tensors with seeds seed0 .. seed0 + count - 1."""
    dev = model.device
    xs = torch.empty(count, model.din, dtype=torch.bfloat16, device=dev)
    tg = torch.empty(count, model.dout, dtype=torch.float32, device=dev)
    t0 = time.time()
    for c0 in range(0, count, chunk):
        n = min(chunk, count - c0)
        Xs, inits = [], []
        for j in range(n):
            seed = seed0 + c0 + j
            X = build_tensor(c5_factors(model.shape, model.R, seed), dev)
            xs[c0 + j] = model.sketch(X)
            Xs.append(X)
            inits.append(synth.init_factors(model.shape, model.R, seed))
        B = C.AlsBatch(Xs, inits, sweeps)
        B.run(sweeps, init=True)
        torch.cuda.synchronize()
        rows = [pack_targets([a.cpu().numpy() for a in B.A[j]], B.lam[j].cpu().numpy()) for j in range(n)]
        tg[c0:c0 + n] = torch.as_tensor(np.stack(rows), device=dev)
        del Xs, B
        log("  dataset %d/%d tensors (%.1f s)" % (c0 + n, count, time.time() - t0))
    return xs, tg


def train(model, xs, tg, epochs, batch=256, lr=1e-3, seed=1, log=print):
    """Adam over shuffled minibatches; returns the mean loss of each epoch."""
    rng = np.random.default_rng(seed)
    n = xs.shape[0] // batch * batch
    hist = []
    for ep in range(epochs):
        perm = torch.as_tensor(rng.permutation(xs.shape[0])[:n], device=xs.device)
        tot = torch.zeros((), dtype=torch.float32, device=xs.device)
        for b0 in range(0, n, batch):
            idx = perm[b0:b0 + batch]
            loss = model.train_step(xs[idx].contiguous(), tg[idx].contiguous(), lr)
            tot += loss.sum()
        hist.append(float(tot) / n)
        log("  epoch %d: mean loss %.4f" % (ep + 1, hist[-1]))
    return hist


def hosvd_start(X, R, seed):
    """Randomized HOSVD start of a device tensor (modes 2 and 3; A_1 is
    never read by Alg. 2 and is returned as zeros), FP64 host arrays."""
    shape = tuple(X.shape)
    Om = [C.colmajor(torch.as_tensor(o, dtype=torch.float64, device=X.device))
          for o in synth.gaussian_factors(shape, R, seed)]
    A = C.cpqr_hosvd_init(X, Om, R, prec=C.PREC_F32, k0=1)
    return [np.zeros((shape[0], R))] + [a.cpu().numpy() for a in A[1:]]


def fit_history(X, init, sweeps):
    """Relative errors (direct form) after each of `sweeps` CP-ALS-QR sweeps
    from `init` and the GPU seconds they took, error included."""
    st = C.AlsState(X, init, prec=C.PREC_F32, error_mode=C.ERROR_DIRECT)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    st.init()
    rel = st.sweep(sweeps)
    e1.record()
    torch.cuda.synchronize()
    return rel.cpu().numpy(), e0.elapsed_time(e1) / 1e3


MARKS = (5, 10, 25, 50, 100, 200)


def summarize(hist, secs, target=1e-6):
    """Relative error at the marked sweep counts, and the sweeps and seconds
    to reach `target` (None when not reached)."""
    hit = next((i + 1 for i, v in enumerate(hist) if v <= target), None)
    return {"relerr_at": {m: float(hist[m - 1]) for m in MARKS if m <= len(hist)},
            "sweeps_to_target": hit, "seconds_to_target": None if hit is None else secs * hit / len(hist),
            "final": float(hist[-1])}


def usable_start(pred, fallback, cond_max=1e8):
    """The predicted factors as a CP-ALS-QR start, or the fallback (HOSVD)
    start when a predicted A_2 or A_3 is non-finite or numerically rank
    deficient.  Returns (factors, used_prediction)."""
    for k in (1, 2):
        a = pred[k]
        if not np.all(np.isfinite(a)) or np.linalg.cond(a) > cond_max:
            return fallback, False
    return pred, True


def evaluate(model, count, seed0, max_sweeps=200, log=print):
    """Held-out tensors (seeds seed0 ..): CP-ALS-QR from the random start,
    the HOSVD start and the learned start (HOSVD when the prediction is not
    usable), the direct relative error after each sweep.  Returns per-tensor
    records (summarize() of each start)."""
    recs = []
    for c0 in range(0, count, 64):
        n = min(64, count - c0)
        sk = torch.zeros(64, model.din, dtype=torch.bfloat16, device=model.device)
        for j in range(n):
            sk[j] = model.sketch(build_tensor(c5_factors(model.shape, model.R, seed0 + c0 + j), model.device))
        preds = model.predict(sk)
        for j in range(n):
            seed = seed0 + c0 + j
            X = build_tensor(c5_factors(model.shape, model.R, seed), model.device)
            rnd = synth.init_factors(model.shape, model.R, seed)
            hos = hosvd_start(X, model.R, seed + 7)
            start, used = usable_start(preds[j], hos)
            rec = {"seed": seed, "used_prediction": used}
            for key, init in (("random", rnd), ("hosvd", hos), ("learned", start)):
                rec[key] = summarize(*fit_history(X, init, max_sweeps))
            recs.append(rec)
            log("  held-out %d: relerr after 10 / 50 / %d sweeps: random %.2e %.2e %.2e, hosvd %.2e %.2e %.2e, "
                "learned %.2e %.2e %.2e" % ((c0 + j, max_sweeps) + tuple(
                    rec[k]["relerr_at"].get(m, float("nan")) for k in ("random", "hosvd", "learned")
                    for m in (10, 50, max_sweeps))))
    return recs


def heldout_loss(model, count, seed0):
    """Mean cosine-form Kruskal loss of the network's prediction against the
    ground-truth factors of held-out tensors (1 - squared cosine between the
    predicted and the true tensor)."""
    sk = torch.zeros(64 * ((count + 63) // 64), model.din, dtype=torch.bfloat16, device=model.device)
    tg = torch.zeros(sk.shape[0], model.dout, dtype=torch.float32, device=model.device)
    for j in range(count):
        A = c5_factors(model.shape, model.R, seed0 + j)
        sk[j] = model.sketch(build_tensor(A, model.device))
        tg[j] = torch.as_tensor(pack_targets(A, np.ones(model.R)), device=model.device)
    y, _ = model.forward(sk)
    loss, _, _ = C.cpqr_kruskal_loss_grad(y, tg, model.shape, model.R, model.R, kind=C.LOSS_COSINE)
    return float(loss[:count].double().mean())
