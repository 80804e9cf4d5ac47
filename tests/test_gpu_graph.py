"""Sweeps captured into a HIP graph (cpqr_als_graph_create) replay exactly
the eager sweeps: after every launch the relative errors, weights and
factors equal, bit for bit, those of the same number of eager sweeps on an
identical state.  Launches are interleaved with other eager work and host
synchronizations, and every launch is checked, not only the last."""

import numpy as np
import pytest
import torch

from paper_2112_10855_amd import cpqr as C
from paper_2112_10855_amd import synth
from helpers import to_dev

pytestmark = pytest.mark.gpu


def same_state(a, b):
    return (torch.equal(a.lam, b.lam) and all(torch.equal(x, y) for x, y in zip(a.A, b.A)))


def check_replays(make, per_launch, launches=4):
    ea, gb = make(), make()
    ea.init()
    gb.init()
    g = gb.graph(per_launch)
    for i in range(launches):
        rel_e = ea.sweep(per_launch).clone()
        rel_g = g.launch().clone()
        # unrelated eager work and a host synchronization between replays
        junk = torch.randn(1000, device="cuda").sum()
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
        assert torch.equal(rel_e, rel_g), (i, rel_e, rel_g)
        assert same_state(ea, gb), i


@pytest.mark.parametrize("per_launch", [1, 3])
@pytest.mark.parametrize("error_mode", [C.ERROR_EFFICIENT, C.ERROR_DIRECT])
def test_graph_dense_fp32_three_way(per_launch, error_mode):
    d = synth.cp_tensor((60, 50, 40), 6, 5, noise=1e-3, dtype=np.float32)
    init = synth.init_factors((60, 50, 40), 6, 6)
    Xd = to_dev(d["X"], torch.float32)
    check_replays(lambda: C.AlsState(Xd, init, prec=C.PREC_F32, error_mode=error_mode), per_launch)


@pytest.mark.parametrize("chain", [0, 1])
def test_graph_dense_fp64_four_way(chain):
    shape = (14, 12, 10, 9)
    d = synth.cp_tensor(shape, 5, 8, noise=1e-3, dtype=np.float64)
    init = synth.init_factors(shape, 5, 9)
    Xd = to_dev(d["X"])
    check_replays(lambda: C.AlsState(Xd, init, prec=C.PREC_F64, krp_chain=chain), 2)


def test_graph_three_way_structured_qr():
    """N = 3 with the structured QR: Q_0 is copied from its single factor
    (a device-to-device copy node in the graph)."""
    shape = (20, 18, 16)
    d = synth.cp_tensor(shape, 4, 10, noise=1e-3, dtype=np.float64)
    init = synth.init_factors(shape, 4, 11)
    Xd = to_dev(d["X"])
    check_replays(lambda: C.AlsState(Xd, init, prec=C.PREC_F64, krp_chain=1), 1)


@pytest.mark.parametrize("solver", ["chol", "pinv"])
def test_graph_normal_equations(solver):
    shape = (40, 30, 35)
    d = synth.cp_tensor(shape, 5, 12, noise=1e-3, dtype=np.float32)
    init = synth.init_factors(shape, 5, 13)
    Xd = to_dev(d["X"], torch.float32)
    check_replays(lambda: C.AlsNeState(Xd, init, prec=C.PREC_F32, solver=solver), 2)


@pytest.mark.parametrize("algo", ["qr", "chol"])
@pytest.mark.parametrize("shape", [(9, 8, 7, 6), (12, 11)])
def test_graph_kruskal_input(algo, shape):
    g = np.random.default_rng(21)
    S, R = 7, 4
    mu = to_dev(g.standard_normal(S))
    V = [to_dev(g.standard_normal((s, S))) for s in shape]
    init = [g.standard_normal((s, R)) for s in shape]
    if algo == "qr":
        make = lambda: C.AlsState(None, init, prec=C.PREC_F64, kruskal=(mu, V))
    else:
        make = lambda: C.AlsNeState(None, init, prec=C.PREC_F64, kruskal=(mu, V))
    check_replays(make, 2)
