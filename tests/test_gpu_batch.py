"""GPU tests of batched replicas (mdpd_create_batch; needs an MI355X).

Replica r of a batch must evolve bit for bit like a system created alone
from its slice of the inputs with its own parameters: the sort key, the
neighbour-list order and every summation order are per replica, and the
noise is keyed on the replica's seed and its local ids.  The standalone path
is itself held to the oracle by test_gpu_parity.py; one replica is also
compared with the oracle directly here.  Every case prints its name first.
"""
import numpy as np
import pytest

import oracle
from paper_1903_10134_amd import workloads as W
from test_gpu_parity import FP64_TOL, dense_cluster, force_err, mixed_types, orc_params, say, small_channel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mdpd():
    import torch
    assert torch.cuda.is_available()
    import paper_1903_10134_amd as m
    m.lib()
    return m


def uneven_replicas():
    """Replicas of uneven size, box shape and parameters, including one that
    overflows the list rows, one with two types and frozen particles, and an
    empty one."""
    reps = W.replicas(count=4, lo=4.0, hi=7.0, seed=3)
    empty = W.bulk(L=4.0, n=0, seed=9)
    return reps + [dense_cluster(), mixed_types(), empty, W.bulk(box=(5.0, 3.5, 8.25), n=700, seed=12)]


def split(arr, offsets):
    return [arr[offsets[r]:offsets[r + 1]] for r in range(len(offsets) - 1)]


@pytest.mark.parametrize("skin", [0.0, 0.3])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_batch_equals_standalone_bitwise(mdpd, prec, skin):
    """With a skin every replica decides its own list rebuilds, so a replica
    in a batch still steps bit for bit like the same system alone."""
    reps = uneven_replicas()
    p = mdpd.FP32_FORCES if prec == "fp32" else mdpd.FP64
    say("batch vs standalone", prec, len(reps), "replicas, skin", skin)
    b = mdpd.Batch(reps, precision=p, skin=skin)
    b.step(6)
    xb, vb, rb = b.state()
    Fb = b.forces()
    ob = b.observables()
    cb, hb = b.neighbors(1.0)
    for r, w in enumerate(reps):
        s = mdpd.System(w, precision=p, skin=skin)
        s.step(6)
        x, v, rho = s.state()
        sl = slice(b.offsets[r], b.offsets[r + 1])
        assert np.array_equal(xb[sl], x), (r, "x")
        assert np.array_equal(vb[sl], v), (r, "v")
        assert np.array_equal(rb[sl], rho), (r, "rho")
        assert np.array_equal(Fb[sl], s.forces()), (r, "F")
        assert ob[r] == s.observables(), r
        c, h = s.neighbors(1.0)
        assert np.array_equal(cb[sl], c) and np.array_equal(hb[sl], h), (r, "neighbours")
        s.close()
    b.close()


def test_batch_replica_matches_oracle(mdpd):
    reps = W.replicas(count=3, lo=5.0, hi=6.0, seed=1)
    say("batch replica vs oracle")
    b = mdpd.Batch(reps)
    b.step(2)
    Fb = b.forces()
    for r, w in enumerate(reps):
        o = oracle.System(orc_params(w), w.x, w.v)
        o.step(2)
        st = o.state()
        sl = slice(b.offsets[r], b.offsets[r + 1])
        assert force_err(Fb[sl], st["F"]) < FP64_TOL, r
    b.close()


def test_batch_with_walls(mdpd):
    reps = [small_channel(seed=3), small_channel(seed=4)]
    say("batch walls")
    b = mdpd.Batch(reps)
    b.step(5)
    xb, vb, _ = b.state()
    for r, w in enumerate(reps):
        s = mdpd.System(w)
        s.step(5)
        x, v, _ = s.state()
        sl = slice(b.offsets[r], b.offsets[r + 1])
        assert np.array_equal(xb[sl], x) and np.array_equal(vb[sl], v), r
        s.close()
    b.close()


def test_batch_with_wall_slip(mdpd):
    """Replicas with their own wall_slip (0.5 and 1) step exactly as the
    same systems alone."""
    reps = [small_channel(seed=5), small_channel(seed=6)]
    for w, sl in zip(reps, (0.5, 1.0)):
        w.wall_slip = sl
    say("batch wall slip")
    b = mdpd.Batch(reps)
    b.step(5)
    xb, vb, _ = b.state()
    ob = b.observables()
    assert sum(o["ncorr_total"] for o in ob) > 0
    for r, w in enumerate(reps):
        s = mdpd.System(w)
        s.step(5)
        x, v, _ = s.state()
        sl = slice(b.offsets[r], b.offsets[r + 1])
        assert np.array_equal(xb[sl], x) and np.array_equal(vb[sl], v), r
        s.close()
    b.close()


def test_batch_with_dissipation_control(mdpd):
    """Replicas with their own fluid-solid dissipation control (eta 1, off,
    0.5) step exactly as the same systems alone."""
    reps = [small_channel(seed=5), small_channel(seed=6), small_channel(seed=7)]
    for w, eta in zip(reps, (1.0, 0.0, 0.5)):
        w.diss_ctrl, w.diss_rho = eta, 6.0
    say("batch dissipation control")
    b = mdpd.Batch(reps)
    b.step(5)
    xb, vb, _ = b.state()
    for r, w in enumerate(reps):
        s = mdpd.System(w)
        s.step(5)
        x, v, _ = s.state()
        sl = slice(b.offsets[r], b.offsets[r + 1])
        assert np.array_equal(xb[sl], x) and np.array_equal(vb[sl], v), r
        s.close()
    b.close()


def test_one_workgroup_sort_equals_the_multi_pass_sort(mdpd):
    """A batch of at least 64 replicas of up to 12,288 particles and 4,096
    cells is sorted by one workgroup per replica; a standalone system, and a
    batch holding one larger replica, take the multi-pass sort.  Replicas
    must step bit for bit as the same systems alone in both batches."""
    small = [W.bulk(L=4.0 + 0.05 * k, seed=21 + k) for k in range(64)]
    big = W.bulk(L=14.0, seed=23)
    assert big.n > 12288
    say("one-workgroup sort vs multi-pass sort")
    alone = []
    for w in small[:3]:
        s = mdpd.System(w)
        s.step(6)
        alone.append(s.state())
        s.close()
    for reps in (small, small + [big]):
        b = mdpd.Batch(reps)
        b.step(6)
        xb, vb, rb = b.state()
        for r, (x, v, rho) in enumerate(alone):
            sl = slice(b.offsets[r], b.offsets[r + 1])
            assert np.array_equal(xb[sl], x) and np.array_equal(vb[sl], v) and np.array_equal(rb[sl], rho), \
                (len(reps), r)
        b.close()


def test_batch_checkpoint_and_limits(mdpd):
    reps = W.replicas(count=3, lo=4.0, hi=5.0, seed=5)
    say("batch checkpoint")
    a = mdpd.Batch(reps)
    a.step(3)
    buf = mdpd.mdpd_save_checkpoint(a.h)
    a.step(4)
    c = mdpd.Batch(reps)
    mdpd.mdpd_load_checkpoint(c.h, buf)
    c.step(4)
    for u, v in zip(a.state(), c.state()):
        assert np.array_equal(u, v)
    assert a.observables() == c.observables()
    with pytest.raises(mdpd.MdpdError):
        mdpd.mdpd_read_observables(a.h)  # several replicas
    with pytest.raises(mdpd.MdpdError):
        c.forward_record(2)  # recording starts at step 0
    with pytest.raises(mdpd.MdpdError):
        mdpd.mdpd_read_replica_observables(a.h, 2, 2)  # out of range
    a.close()
    c.close()


def test_autotune_leaves_no_trace(mdpd):
    """The tuner restores the state it started from: tuning then stepping
    equals stepping a fresh system with the chosen lanes, bit for bit; the
    second call on the same shape hits the cache."""
    reps = W.replicas(count=3, lo=5.0, hi=6.0, seed=8)
    say("autotune batch")
    a = mdpd.Batch(reps, precision=mdpd.FP32_FORCES)
    a.step(2)
    lanes = a.autotune(steps=2)
    assert all(l in (1, 2, 4, 8, 16) for l in lanes)
    a.step(3)
    b = mdpd.Batch(reps, precision=mdpd.FP32_FORCES)
    b.step(2)
    for k, l in enumerate(lanes):
        b.set_lanes(k, l)
    b.step(3)
    for u, v in zip(a.state(), b.state()):
        assert np.array_equal(u, v)
    assert a.observables() == b.observables()
    assert b.autotune(steps=2) == lanes
    a.close()
    b.close()


@pytest.mark.parametrize("avg", [False, True])
def test_batch_adjoint_equals_standalone(mdpd, avg):
    """Per-replica losses and gradients of a batch equal, bit for bit, those
    of each replica recorded and differentiated alone."""
    reps = W.replicas(count=3, lo=4.0, hi=6.0, seed=4) + [mixed_types(), dense_cluster()]
    say("batch adjoint", "avg" if avg else "final")
    rng = np.random.default_rng(3)
    w = rng.normal(size=(len(reps), 3))
    b = mdpd.Batch(reps, precision=mdpd.FP32_FORCES)
    lb = b.forward_record(5, every=2, average=avg)
    gb = b.backward(w)
    for r, wl in enumerate(reps):
        s = mdpd.System(wl, precision=mdpd.FP32_FORCES)
        ls = s.forward_record(5, every=2, average=avg)
        gs = s.backward(w[r])
        assert np.array_equal(lb[r], ls), r
        sl = slice(b.offsets[r], b.offsets[r + 1])
        for key in ("dA", "dB", "dgamma"):
            assert np.array_equal(gb[key][r], gs[key]), (r, key)
        assert np.array_equal(gb["dx0"][sl], gs["dx0"]), r
        assert np.array_equal(gb["dv0"][sl], gs["dv0"]), r
        s.close()
    b.close()
