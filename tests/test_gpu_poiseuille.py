"""Plane Poiseuille flow between frozen walls (needs an MI355X).

A channel of width 12 (fluid y in [0, 12), frozen slabs of thickness 2 on
both sides, box 16 x 16 x 8, density 6, g_x = 0.02, bounce-back walls) is
driven to its steady state and the fluid velocity, temperature and density
are averaged across the channel in bins of 0.5.  The textbook solution of
the driven plane channel is a parabola in y with its zeros at the walls
(Sec. 2.2: no-slip walls with negligible near-wall density and temperature
fluctuations):

* the mean u_x profile fits a parabola with R^2 > 0.99, opening downward,
  whose zeros lie within 0.5 of the wall planes y = 0 and y = 12;
* the kinetic temperature of the velocities relative to the bin mean stays
  within 2% of kT = 1 in every bin, next to the walls too;
* the density is flat to 2% away from the walls and dips by less than 10% in
  the half-width bins touching them.
Measured: R^2 0.9985, zeros at 0.18 and 11.81, kT 0.999 .. 1.005, density
5.94 inside and 5.52 / 5.60 in the wall bins.  A more attractive wall
(A_SL = -50) flattens the wall bins to within 3% (the second test).
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


def test_poiseuille_profile(mdpd):
    w = W.channel(Lx=16.0, Ly=12.0, Lz=8.0, wall=2.0, gx=0.02, seed=11)
    say("poiseuille", w.n)
    s = mdpd.System(w, precision=mdpd.FP32_FORCES)
    s.step(20000)
    nb = 32                      # bins of 0.5 over the periodic height 16: fluid in bins 0..23
    acc = {q: np.zeros(nb) for q in (0, 1, 4)}
    m = 0
    for _ in range(1000):
        s.step(20)
        for q in acc:
            acc[q] += s.profile(1, nb, q)
        m += 1
    s.close()
    y = (np.arange(24) + 0.5) * 0.5
    u = acc[1][:24] / m
    kt = acc[4][:24] / m
    rho = acc[0][:24] / m
    c = np.polyfit(y, u, 2)
    fit = np.polyval(c, y)
    r2 = 1.0 - np.sum((u - fit) ** 2) / np.sum((u - u.mean()) ** 2)
    roots = np.sort(np.roots(c).real)
    print(f"\nu_x: " + " ".join(f"{v:.3f}" for v in u))
    print(f"kT:  " + " ".join(f"{v:.3f}" for v in kt))
    print(f"rho: " + " ".join(f"{v:.2f}" for v in rho))
    print(f"parabola R^2 {r2:.4f}, zeros at {roots[0]:.3f} and {roots[1]:.3f}, u_max {u.max():.3f}")
    assert c[0] < 0.0
    assert r2 > 0.99
    assert abs(roots[0] - 0.0) < 0.5 and abs(roots[1] - 12.0) < 0.5
    assert np.all(np.abs(kt - 1.0) < 0.02)
    inner = rho[1:23]
    assert np.all(np.abs(inner / inner.mean() - 1.0) < 0.02)
    assert rho[0] > 0.9 * inner.mean() and rho[23] > 0.9 * inner.mean()


def test_neutral_wall_keeps_the_density_flat(mdpd):
    """The same channel with the wall-fluid attraction A_SL = -50 (the fluid's
    own A is -40): the frozen wall then holds the fluid next to it at the bulk
    density, flat to 3% in every bin including the two touching the walls
    (with A_SL = A the wall bins dip 6-7%, see above), while the flow stays
    the no-slip parabola.  Sec. 2.2 asks for negligible near-wall density
    fluctuations and Sec. 4.2 sets A_SL per wall to control the wetting; this
    is the neutral choice for walls of frozen particles at the fluid density.
    Measured: wall bins 5.78 and 5.85 against 5.86 inside, R^2 0.997."""
    w = W.channel(Lx=16.0, Ly=12.0, Lz=8.0, wall=2.0, gx=0.02, seed=11)
    A = np.array(w.A, dtype=float)
    A[0, 1] = A[1, 0] = -50.0
    w.A = A
    say("poiseuille neutral wall", w.n)
    s = mdpd.System(w, precision=mdpd.FP32_FORCES)
    s.step(10000)
    nb = 32
    acc = {q: np.zeros(nb) for q in (0, 1)}
    m = 0
    for _ in range(500):
        s.step(20)
        for q in acc:
            acc[q] += s.profile(1, nb, q)
        m += 1
    s.close()
    y = (np.arange(24) + 0.5) * 0.5
    u = acc[1][:24] / m
    rho = acc[0][:24] / m
    c = np.polyfit(y, u, 2)
    fit = np.polyval(c, y)
    r2 = 1.0 - np.sum((u - fit) ** 2) / np.sum((u - u.mean()) ** 2)
    roots = np.sort(np.roots(c).real)
    print(f"\nrho: " + " ".join(f"{v:.2f}" for v in rho))
    print(f"parabola R^2 {r2:.4f}, zeros at {roots[0]:.3f} and {roots[1]:.3f}")
    assert np.all(np.abs(rho / rho.mean() - 1.0) < 0.03)
    assert c[0] < 0.0 and r2 > 0.99
    assert abs(roots[0] - 0.0) < 0.5 and abs(roots[1] - 12.0) < 0.5
