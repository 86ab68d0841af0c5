"""The control of the effective fluid-solid dissipation in a walled channel
(Sec. 2.2; needs an MI355X).

A fluid particle's fluid-solid pairs take gamma s_i and sigma sqrt(s_i),
with s_i bringing its dissipative weight from the solid to eta rho_f W_D
phi_i (diss_ctrl = eta, diss_rho = rho_f).  Parity with the oracle is in
test_gpu_parity.py; here the physics the control is for:

1. The thermostat stays consistent next to the walls: the random force on a
   fluid-solid pair scales with sqrt(s_i) when its dissipation scales with
   s_i, so a channel at rest keeps kT flat across every bin, the wall bins
   included, for a weak (eta = 0.3) and a strong (eta = 3) control.
2. In a driven channel with bounce-back walls the fluid flows and keeps
   kT flat next to the walls under a weak and a strong control.
"""
import numpy as np
import pytest

from paper_1903_10134_amd import workloads as W
from test_gpu_parity import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mdpd():
    import torch
    assert torch.cuda.is_available()
    import paper_1903_10134_amd as m
    m.lib()
    return m


def profiles(mdpd, eta, gx, steps=4000, sample=8000, every=20):
    w = W.channel(Lx=16.0, Ly=12.0, Lz=8.0, wall=2.0, gx=gx, seed=5)
    w.diss_ctrl, w.diss_rho = eta, 6.0
    say("channel with dissipation control", eta, gx)
    s = mdpd.System(w, precision=mdpd.FP32_FORCES)
    s.step(steps)
    nb = 16  # bins of 1 along y over the periodic height 16: fluid in bins 0..11
    u, kt = np.zeros(nb), np.zeros(nb)
    m = 0
    for _ in range(sample // every):
        s.step(every)
        u += s.profile(1, nb, 1)
        kt += s.profile(1, nb, 4)
        m += 1
    s.close()
    return u[:12] / m, kt[:12] / m


def test_control_keeps_the_thermostat(mdpd):
    for eta in (0.3, 3.0):
        _, kt = profiles(mdpd, eta, 0.0)
        print(f"\neta {eta}: kT " + " ".join(f"{v:.3f}" for v in kt))
        assert np.all(np.abs(kt - 1.0) < 0.02), (eta, kt)


def test_control_in_a_driven_channel(mdpd):
    """Driven channel with bounce-back walls, weak and strong control: the
    fluid flows (u_x > 0 in every bin) and every bin, the wall bins included,
    stays within 2% of kT.  The wall-bin velocities are printed: with the
    bounce-back corrector, whose velocity reversal already holds the fluid
    at the wall, the control changes them by less than their noise."""
    for eta in (0.3, 3.0):
        u, kt = profiles(mdpd, eta, 0.02)
        print(f"\neta {eta}: u_x " + " ".join(f"{v:.3f}" for v in u) + f"  (mean {u.mean():.4f})")
        print(f"eta {eta}: kT  " + " ".join(f"{v:.3f}" for v in kt))
        assert np.all(u > 0.0), (eta, u)
        assert np.all(np.abs(kt - 1.0) < 0.02), (eta, kt)
