"""GPU parity of the adjoint (mdpd_forward_record / mdpd_backward) against the
oracle's forward-mode derivative (needs an MI355X).

The gradient g returned by the reverse pass and the oracle's tangent dL along
a direction d must agree: <g, d> = dL.  Directions: a symmetric unit change
of each pair table, random directions in the initial positions and
velocities.  Bars: FP64 form within 1e-8 relative (the two accumulate the
same derivative in different orders over several steps), FP32-forces form
within 1e-4 relative (its trajectory itself differs at FP32 rounding).
The walled case differentiates the bounce-back corrector with its events
held fixed (the corrected particles' drift is reverted, their half-step
velocity negated), against the oracle's tangent of the same events.
Every case prints its name first so that a failing run names it.
"""
import numpy as np
import pytest

import oracle
from paper_1903_10134_amd import workloads as W
from test_gpu_parity import dense_cluster, mixed_types, orc_params, say

pytestmark = pytest.mark.gpu

LOSSES = {"rho": (1.0, 0.0, 0.0), "pressure": (0.0, 1.0, 0.0), "vx": (0.0, 0.0, 1.0)}


@pytest.fixture(scope="module")
def mdpd():
    import torch
    assert torch.cuda.is_available()
    import paper_1903_10134_amd as m
    m.lib()
    return m


def adj_cases():
    return {
        "bulk_L6": W.bulk(L=6.0, density=6.0, seed=3),
        "mixed_types": mixed_types(),
        "dense_cluster": dense_cluster(),
        # bounce-back walls: the corrector's events of the recorded
        # trajectory are held fixed on both sides
        "channel_walls": W.channel(Lx=6.0, Ly=4.0, Lz=6.0, wall=1.5, seed=3, gx=0.05),
        # the same channel with the fluid-solid dissipation control: the
        # factor s_i of a fluid particle depends on its neighbours' positions
        "channel_walls_dc": dc_channel(),
    }


def dc_channel():
    w = W.channel(Lx=6.0, Ly=4.0, Lz=6.0, wall=1.5, seed=3, gx=0.05)
    w.diss_ctrl, w.diss_rho = 0.8, 6.0
    w.name = "channel_walls_dc"
    return w


CASES = adj_cases()


def table_dirs(T):
    """Symmetric unit directions of a T x T table: (a, b) with a <= b."""
    out = []
    for a in range(T):
        for b in range(a, T):
            E = np.zeros((T, T))
            E[a, b] = E[b, a] = 1.0
            out.append(((a, b), E))
    return out


def check(mdpd, w, prec, nsteps, every, avg, tol, skin=None):
    p = mdpd.FP32_FORCES if prec == "fp32" else mdpd.FP64
    op = orc_params(w)
    s = mdpd.System(w, precision=p, skin=skin)
    loss = s.forward_record(nsteps, every=every, average=avg)
    n = w.x.shape[0]
    T = np.atleast_2d(w.A).shape[0]
    rng = np.random.default_rng(nsteps + 3)
    dx = rng.standard_normal((n, 3))
    dv = rng.standard_normal((n, 3))
    for lname, wts in LOSSES.items():
        gr = s.backward(wts)
        L_o, _ = oracle.tangent(op, w.x, w.v, w.types, w.frozen, nsteps, wts, avg)
        # the FP32 form does not conserve momentum exactly (f_ij and f_ji are
        # rounded separately), so the mean velocity drifts at FP32 rounding
        floor = 1e-11 if prec == "fp64" else 1e-6
        assert float(np.dot(loss, wts)) == pytest.approx(L_o, rel=max(tol, 1e-11), abs=floor), lname
        checks = [("x0", float(np.sum(gr["dx0"] * dx)), dict(dx0=dx)),
                  ("v0", float(np.sum(gr["dv0"] * dv)), dict(dv0=dv))]
        for (a, b), E in table_dirs(T):
            for key, name in (("dA", "A"), ("dB", "B"), ("dgamma", "gamma")):
                checks.append((f"{name}[{a},{b}]", float(np.sum(gr[key] * E)), {key: E.ravel()}))
        for what, val, kw in checks:
            _, ref = oracle.tangent(op, w.x, w.v, w.types, w.frozen, nsteps, wts, avg, **kw)
            scale = max(abs(ref), 1e-3 if lname != "pressure" else 1e-1)
            assert abs(val - ref) <= tol * scale, (lname, what, val, ref)
    s.close()


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("avg", [False, True])
def test_adjoint_matches_oracle_tangent_fp64(mdpd, name, avg):
    say("adjoint fp64", name, "avg" if avg else "final")
    check(mdpd, CASES[name], "fp64", nsteps=5, every=2, avg=avg, tol=1e-8)


@pytest.mark.parametrize("name", ["bulk_L6", "channel_walls"])
def test_adjoint_with_skin_list(mdpd, name):
    """A skin list (rebuilt only when particles have moved half the skin)
    records the same trajectory and so the same derivative."""
    say("adjoint fp64 skin", name)
    check(mdpd, CASES[name], "fp64", nsteps=8, every=3, avg=True, tol=1e-8, skin=0.3)


def test_adjoint_fp32_form(mdpd):
    say("adjoint fp32 bulk_L6")
    check(mdpd, CASES["bulk_L6"], "fp32", nsteps=4, every=3, avg=True, tol=1e-4)


def test_adjoint_zero_steps(mdpd):
    say("adjoint nsteps=0")
    check(mdpd, CASES["mixed_types"], "fp64", nsteps=0, every=1, avg=False, tol=1e-9)


def test_adjoint_independent_of_checkpoint_spacing(mdpd):
    """Recomputation reproduces the recorded trajectory bit for bit, so the
    gradient does not depend on the checkpoint spacing."""
    w = CASES["bulk_L6"]
    say("adjoint every", w.name)
    res = []
    for every in (1, 3, 7, 100):
        s = mdpd.System(w, precision=mdpd.FP32_FORCES)
        s.forward_record(7, every=every, average=True)
        res.append(s.backward((0.7, 0.01, -2.0)))
        s.close()
    for r in res[1:]:
        for k in r:
            assert np.array_equal(r[k], res[0][k]), k


def test_adjoint_leaves_state_at_end_of_recording(mdpd):
    w = CASES["bulk_L6"]
    say("adjoint restores state")
    a = mdpd.System(w)
    a.forward_record(6, every=4)
    a.backward((1.0, 0.0, 0.0))
    a.step(3)
    b = mdpd.System(w)
    b.step(9)
    for u, v in zip(a.state(), b.state()):
        assert np.array_equal(u, v)
    assert a.observables() == b.observables()
    a.close()
    b.close()


def test_adjoint_errors(mdpd):
    w = CASES["bulk_L6"]
    say("adjoint errors")
    s = mdpd.System(w)
    with pytest.raises(mdpd.MdpdError):
        s.backward((1.0, 0.0, 0.0))  # nothing recorded
    with pytest.raises(mdpd.MdpdError):
        s.forward_record(0, average=True)
    s.step(1)
    with pytest.raises(mdpd.MdpdError):
        s.forward_record(3)  # not at step 0
    s.close()
    from test_gpu_parity import small_channel
    w = small_channel()
    w.wall_slip = 0.5
    c = mdpd.System(w)
    with pytest.raises(mdpd.MdpdError):
        c.forward_record(2)  # reflecting walls
    c.close()


@pytest.mark.parametrize("name", ["mixed_types", "channel_walls"])
def test_autograd_function(mdpd, name):
    """torch.autograd: loss.backward() fills the gradients of x0, v0, A, B,
    gamma with what mdpd_backward returns for the same upstream weights."""
    import torch
    from paper_1903_10134_amd.autograd import trajectory_loss
    w = CASES[name]
    say("autograd", w.name)
    dev = torch.device("cuda")
    x0 = torch.tensor(w.x, device=dev, requires_grad=True)
    v0 = torch.tensor(w.v, device=dev, requires_grad=True)
    A = torch.tensor(np.atleast_2d(w.A), requires_grad=True)
    B = torch.tensor(np.atleast_2d(w.B), requires_grad=True)
    G = torch.tensor(np.atleast_2d(w.gamma), requires_grad=True)
    kw = w.param_kwargs()
    out = trajectory_loss(x0, v0, A, B, G, torch.tensor(w.types), torch.tensor(w.frozen), kw["box"], nsteps=4,
                          every=2, average=True, rc=kw["rc"], rd=kw["rd"], kT=kw["kT"], dt=kw["dt"],
                          mass=kw["mass"], g=kw["g"], seed=kw["seed"], wall_model=kw["wall_model"],
                          phi_c=kw["phi_c"])
    wts = (0.5, 0.02, -1.0)
    (out * torch.tensor(wts, dtype=torch.float64, device=dev)).sum().backward()
    s = mdpd.System(w)
    ref_loss = s.forward_record(4, every=2, average=True)
    ref = s.backward(wts)
    s.close()
    assert np.array_equal(out.detach().cpu().numpy(), ref_loss)
    assert np.array_equal(x0.grad.cpu().numpy(), ref["dx0"])
    assert np.array_equal(v0.grad.cpu().numpy(), ref["dv0"])
    assert np.array_equal(A.grad.numpy(), ref["dA"])
    assert np.array_equal(B.grad.numpy(), ref["dB"])
    assert np.array_equal(G.grad.numpy(), ref["dgamma"])


def test_batched_adjoint_long_horizon_and_finite_differences(mdpd):
    """The batched workload shape (uneven periodic replicas, per-replica A
    and B), checkpoints every 10 steps, time-averaged mean density and
    pressure.  Over 100 steps the adjoint equals the oracle's forward-mode
    derivative of the same loss (the exact derivative of the discrete
    trajectory).  Finite differences of the GPU's own FP64 losses are checked
    over 20 steps: over 100 steps pairs crossing the cutoffs, where the force
    derivative jumps, make them converge slowly in h (at h = 1e-3, 1e-4, 1e-6
    they are 21%, 9% and 0.2% off the exact derivative for replica 0)."""
    reps = W.replicas(count=3, lo=6.0, hi=7.0, seed=11)
    say("batched adjoint, 100 steps vs oracle tangent", [r.n for r in reps])
    wts = np.tile([1.0, 0.05, 0.0], (len(reps), 1))
    b = mdpd.Batch(reps)
    b.forward_record(100, every=10, average=True)
    g = b.backward(wts)
    b.close()
    for r in (0, 1):
        wr = reps[r]
        op = orc_params(wr, search=1)
        for gk in ("dA", "dB", "dgamma"):
            _, tan = oracle.tangent(op, wr.x, wr.v, wr.types, wr.frozen, 100, wts[r], True, **{gk: [1.0]})
            assert abs(float(g[gk][r][0, 0]) - tan) <= 1e-6 * abs(tan) + 1e-10, (r, gk, g[gk][r], tan)

    say("batched adjoint, 20 steps vs finite differences")
    b = mdpd.Batch(reps)
    b.forward_record(20, every=10, average=True)
    g = b.backward(wts)
    b.close()

    def loss(key, r, eps):
        reps2 = W.replicas(count=3, lo=6.0, hi=7.0, seed=11)
        setattr(reps2[r], key, np.atleast_2d(getattr(reps2[r], key)) + eps)
        bb = mdpd.Batch(reps2)
        L = bb.forward_record(20, every=20, average=True)
        bb.close()
        return float(np.dot(L[r], wts[r]))

    h = 1e-6  # a pair crossing a cutoff within +-h spoils a difference; that chance grows with h
    for r in range(len(reps)):
        for key, gk in (("A", "dA"), ("B", "dB"), ("gamma", "dgamma")):
            fd = (loss(key, r, h) - loss(key, r, -h)) / (2 * h)
            ad = float(g[gk][r][0, 0])
            assert abs(ad - fd) <= 1e-5 * abs(fd) + 1e-8, (r, key, ad, fd)
