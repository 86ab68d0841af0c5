"""Wall corrector with partial and full slip (Sec. 2.2; needs an MI355X).

A rejected step reflects the half-step velocity about the wall normal
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


def wall_layer_velocity(mdpd, slip, steps=4000, sample=8000, every=20):
    w = W.channel(Lx=16.0, Ly=12.0, Lz=8.0, wall=2.0, gx=0.02, seed=2)
    w.wall_slip = slip
    w.gamma = np.array([[4.5, 0.0], [0.0, 4.5]])
    say("channel slip flow", slip)
    s = mdpd.System(w, precision=mdpd.FP32_FORCES)
    s.step(steps)
    nb = 16  # bins of 1 along y over the periodic height 16: fluid in bins 0..11
    ux = np.zeros(nb)
    m = 0
    for _ in range(sample // every):
        s.step(every)
        ux += s.profile(1, nb, 1)
        m += 1
    s.close()
    return ux[:12] / m


def test_full_slip_speeds_up_the_wall_layer(mdpd):
    u0 = wall_layer_velocity(mdpd, 0.0)
    u1 = wall_layer_velocity(mdpd, 1.0)
    print("\nu_x across the channel, bounce-back: " + " ".join(f"{u:.3f}" for u in u0))
    print("u_x across the channel, full slip:   " + " ".join(f"{u:.3f}" for u in u1))
    wall0 = 0.5 * (u0[0] + u0[-1])
    wall1 = 0.5 * (u1[0] + u1[-1])
    assert np.all(u0 > 0.0) and np.all(u1 > 0.0)
    assert wall1 > wall0
