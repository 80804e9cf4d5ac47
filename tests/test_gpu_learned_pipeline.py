"""The learned-initialization pipeline end to end at a small size: method
targets from the batched CP-ALS-QR, training on the GPU kernels, and the
prediction used as a CP-ALS-QR start.  What the trained network gains over
the untrained one on held-out tensors is measured and printed; training is
required to lower the training loss (the kernels and Adam work together)."""

import numpy as np
import pytest
import torch

from paper_2112_10855_amd import learned as LI

pytestmark = pytest.mark.gpu


def test_pipeline_trains_and_initializes():
    model = LI.LearnedInit(shape=(64, 64, 64), R=4, J=64, hidden=64, seed=3)
    xs, tg = LI.make_dataset(model, 256, seed0=500, sweeps=30, chunk=128, log=lambda *a: None)
    assert torch.isfinite(tg).all()
    before = LI.heldout_loss(model, 64, 9000)
    hist = LI.train(model, xs, tg, epochs=15, batch=64, lr=1e-3, log=lambda *a: None)
    after = LI.heldout_loss(model, 64, 9000)
    print("train loss %.4f -> %.4f, held-out %.4f -> %.4f" % (hist[0], hist[-1], before, after))
    assert hist[-1] < hist[0]
    assert np.isfinite(after)
    recs = LI.evaluate(model, 2, 9000, max_sweeps=60, log=lambda *a: None)
    for r in recs:
        assert r["learned"][2] == r["learned"][2]  # a finite relative error came back
