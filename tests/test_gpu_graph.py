"""GPU tests of graph mode (mdpd_set_graph; needs an MI355X): replaying the
captured pair of timesteps gives bit for bit the trajectory of eager
stepping, across several replays with eager work and synchronisations in
between, odd step counts, walls, a batch, a lane change (recapture) and a
checkpoint load that changes the buffer parity.  Every case prints its name.
"""
import numpy as np
import pytest

from paper_1903_10134_amd import workloads as W
from test_gpu_parity import CASES, say, small_channel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mdpd():
    import torch
    assert torch.cuda.is_available()
    import paper_1903_10134_amd as m
    m.lib()
    return m


def same(a, b):
    for u, v in zip(a.state(), b.state()):
        assert np.array_equal(u, v)
    assert np.array_equal(a.forces(), b.forces())


@pytest.mark.parametrize("skin", [0.0, 0.3])
@pytest.mark.parametrize("case", ["bulk_L10_n6000", "mixed_types", "small_channel"])
def test_graph_equals_eager(mdpd, case, skin):
    """Replays equal eager stepping bit for bit; with a skin the list
    rebuilds are decided on the device inside the replays too."""
    w = small_channel() if case == "small_channel" else CASES[case]
    say("graph", case, "skin", skin)
    g = mdpd.System(w, precision=mdpd.FP32_FORCES, skin=skin)
    e = mdpd.System(w, precision=mdpd.FP32_FORCES, skin=skin)
    g.set_graph(True)
    for chunk in (4, 3, 6, 1, 2):  # replays, odd remainders run eagerly
        g.step(chunk)
        e.step(chunk)
        same(g, e)
        assert g.observables() == e.observables()
    g.close()
    e.close()


def test_graph_recapture_on_lanes_and_parity(mdpd):
    w = CASES["bulk_L10_n6000"]
    say("graph recapture")
    g = mdpd.System(w)
    e = mdpd.System(w)
    g.set_graph(True)
    g.step(4)
    e.step(4)
    for s in (g, e):
        s.set_lanes(2, 8)
    g.step(4)
    e.step(4)
    same(g, e)
    buf = e.save_checkpoint()
    e.step(1)  # one eager step flips the buffer parity: the next replay recaptures
    g.step(1)
    g.load_checkpoint(buf)
    e.load_checkpoint(buf)
    g.step(6)
    e.step(6)
    same(g, e)
    g.set_graph(False)
    g.step(2)
    e.step(2)
    same(g, e)
    g.close()
    e.close()


def test_graph_batch(mdpd):
    reps = W.replicas(count=5, lo=4.0, hi=6.0, seed=2)
    say("graph batch")
    g = mdpd.Batch(reps)
    e = mdpd.Batch(reps)
    g.set_graph(True)
    g.step(8)
    e.step(8)
    same(g, e)
    assert g.observables() == e.observables()
    g.close()
    e.close()
