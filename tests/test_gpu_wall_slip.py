"""Wall corrector with partial and full slip (Sec. 2.2; needs an MI355X).

A rejected step reflects the velocity about the wall normal
n = unit(sum_{frozen j, r<r_c} w_c^2 (x_i - x_j) / r): normal part negated,
tangential part times 2 wall_slip - 1 (0: bounce-back, 1: specular).

1. The closed form of the flat-lattice case the oracle is pinned to.
2. Parity of the walled two-type step against the oracle for wall_slip 0.5
   and 1 (corrector counts step by step, FP64 positions and forces).
3. The flow it is for: in a driven channel whose fluid-wall pairs have no
   dissipative (and so no random) force, the fluid next to the walls moves
   faster with full slip than with bounce-back, which holds it back.
"""
import numpy as np
import pytest

import oracle
from paper_1903_10134_amd import workloads as W
from test_gpu_parity import force_err, orc_params, pdiff, say
from test_oracle_pins import wall_and_particle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mdpd():
    import torch
    assert torch.cuda.is_available()
    import paper_1903_10134_amd as m
    m.lib()
    return m


@pytest.mark.parametrize("slip", [0.0, 0.25, 0.5, 1.0])
def test_flat_wall_reflection(mdpd, slip):
    v0 = np.array([1.0, -1.0, 1.0])
    _, x, v, t, f = wall_and_particle(oracle, slip, v0)
    say("flat wall reflection", slip)
    p = mdpd.make_params(box=8.0, A=0.0, B=0.0, gamma=0.0, kT=0.0, dt=0.0625, wall_model=1, phi_c=0.5,
                         wall_slip=slip)
    s = mdpd.System(params=p, x=x, v=v, types=t, frozen=f)
    s.step(1)
    xs, vs, _ = s.state()
    assert s.observables()["ncorr_last"] == 1
    assert np.array_equal(xs[0], x[0])
    if slip == 0.0:
        assert np.array_equal(vs[0], -v0)
    else:
        assert np.allclose(vs[0], [2 * slip - 1, 1.0, 2 * slip - 1], atol=1e-12, rtol=0)
    s.close()


@pytest.mark.parametrize("slip", [0.0, 0.25, 0.5, 1.0])
def test_flat_wall_reflection_with_a_tangential_kick(mdpd, slip):
    """The oracle's closed form with a body force along the wall: the
    rejected step ends at R v_half + k (the normal kick cancels)."""
    k = np.array([1.0 / 128.0, 0.0, 1.0 / 64.0])
    v0 = np.array([1.0, -1.0, 1.0]) - k
    _, x, v, t, f = wall_and_particle(oracle, slip, v0, g=(0.25, 0.0, 0.5))
    say("flat wall reflection with a kick", slip)
    p = mdpd.make_params(box=8.0, A=0.0, B=0.0, gamma=0.0, kT=0.0, dt=0.0625, wall_model=1, phi_c=0.5,
                         wall_slip=slip, g=(0.25, 0.0, 0.5))
    s = mdpd.System(params=p, x=x, v=v, types=t, frozen=f)
    s.step(1)
    xs, vs, _ = s.state()
    assert s.observables()["ncorr_last"] == 1
    assert np.array_equal(xs[0], x[0])
    ft = 2.0 * slip - 1.0
    exp = np.array([ft + k[0], 1.0, ft + k[2]]) if slip > 0.0 else -v0
    assert np.allclose(vs[0], exp, atol=1e-15, rtol=0), (vs[0], exp)
    s.close()


@pytest.mark.parametrize("slip", [0.25, 1.0])
def test_reflection_twice_in_a_row_bounces_back(mdpd, slip):
    """The oracle's closed form: a particle held against the wall is
    reflected at its first rejection and bounced back at every later one."""
    v0 = np.array([1.0, 0.0, 1.0])
    _, x, v, t, f = wall_and_particle(oracle, slip, v0, g=(0.0, -0.5, 0.0))
    say("reflection twice in a row", slip)
    p = mdpd.make_params(box=8.0, A=0.0, B=0.0, gamma=0.0, kT=0.0, dt=0.0625, wall_model=1, phi_c=0.5,
                         wall_slip=slip, g=(0.0, -0.5, 0.0))
    s = mdpd.System(params=p, x=x, v=v, types=t, frozen=f)
    ft = 2.0 * slip - 1.0
    v1 = np.array([ft, 0.0, ft])
    for k, exp in enumerate((v1, -v1, v1, -v1)):
        s.step(1)
        xs, vs, _ = s.state()
        assert s.observables()["ncorr_last"] == 1, k
        assert np.array_equal(xs[0], x[0]), k
        assert np.allclose(vs[0], exp, atol=1e-15, rtol=0), (k, vs[0], exp)
    s.close()


@pytest.mark.parametrize("slip", [0.5, 1.0])
def test_slip_parity_fp64(mdpd, slip):
    w = W.slit_pore(A_SL=-35.0, seed=1)
    w.wall_slip = slip
    say("slit pore slip parity", slip)
    s = mdpd.System(w, precision=mdpd.FP64)
    o = oracle.System(orc_params(w, search=1), w.x, w.v, w.types, w.frozen)
    total = 0
    for k in range(8):
        s.step(1)
        o.step(1)
        a, b = s.observables(), o.observables()
        assert a["ncorr_last"] == b["ncorr_last"], (k, a["ncorr_last"], b["ncorr_last"])
        total += b["ncorr_last"]
    st = o.state()
    x, v, _ = s.state()
    assert total > 0
    assert pdiff(x, st["x"], w.box) < 1e-10
    assert np.max(np.abs(v - st["v"])) < 1e-10
    assert force_err(s.forces(), st["F"]) < 1e-10
    s.close()


def channel_profiles(mdpd, slip, steps=4000, sample=8000, every=20):
    """u_x and kT across a driven channel whose fluid-wall pairs have no
    dissipative (and so no random) force, in bins of 1 over the fluid."""
    w = W.channel(Lx=16.0, Ly=12.0, Lz=8.0, wall=2.0, gx=0.02, seed=2)
    w.wall_slip = slip
    w.gamma = np.array([[4.5, 0.0], [0.0, 4.5]])
    say("channel slip flow", slip)
    s = mdpd.System(w, precision=mdpd.FP32_FORCES)
    s.step(steps)
    nb = 16  # bins of 1 along y over the periodic height 16: fluid in bins 0..11
    ux, kt = np.zeros(nb), np.zeros(nb)
    m = 0
    for _ in range(sample // every):
        s.step(every)
        ux += s.profile(1, nb, 1)
        kt += s.profile(1, nb, 4)
        m += 1
    s.close()
    return ux[:12] / m, kt[:12] / m


def test_slip_channel_flow_and_temperature(mdpd):
    """The fluid flows with every reflection (u_x > 0 off the wall bins,
    mean above 0.1).  Bounce-back and full slip keep every bin, the wall
    bins included, at the bulk temperature: a particle sent back again in
    the step after a reflection is bounced back, so it cannot stay at the
    wall taking the step's tangential impulse without moving (which ran the
    wall bins at kT 2.5 to 3 before that rule).  Half slip drops the
    tangential velocity of a corrected particle, which can only cool the
    wall bins.  Next to the walls full slip lets the fluid move faster than
    bounce-back, which holds it back."""
    rows = {}
    for slip in (0.0, 0.5, 1.0):
        u, kt = channel_profiles(mdpd, slip)
        rows[slip] = u
        print(f"\nslip {slip}: u_x " + " ".join(f"{v:.3f}" for v in u) + f"  (mean {u.mean():.4f})")
        print(f"slip {slip}: kT  " + " ".join(f"{v:.3f}" for v in kt))
        assert np.all(u[1:-1] > 0.0) and u.mean() > 0.1, (slip, u)
        if slip in (0.0, 1.0):
            assert np.all(np.abs(kt - 1.0) < 0.05), (slip, kt)
        else:
            assert np.all(kt < 1.05) and np.all(np.abs(kt[2:-2] - 1.0) < 0.05), (slip, kt)
    wall0 = 0.5 * (rows[0.0][0] + rows[0.0][-1])
    wall1 = 0.5 * (rows[1.0][0] + rows[1.0][-1])
    assert wall1 > wall0, (wall0, wall1)
