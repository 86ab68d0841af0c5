"""Sec. 4.2, static contact angle of one fluid in a slit nano channel (needs
an MI355X).

Set-up: ``workloads.slit_pore`` (60 x 10 x 5 box, 3,500 frozen wall
particles in two layers of thickness r_c, 4,000 fluid particles, boundary-
volume-fraction walls).  The paper's parameter table puts the three varied
values in the liquid-liquid cell while its text varies the solid-liquid
parameter; the text is followed: A_SS = A_LL = -40, A_SL in {-35, -30, -20},
B = 25 and r_d = 0.75 for every pair.

1. Parity: the first steps of the A_SL = -35 case against the oracle
   (identical corrector counts step by step; FP64 positions and forces).
2. The wetting trend the text reports, as qualitative pins: after 4,000
   steps the number of fluid particles in eight bins across the pore width is
   averaged over 10,000 steps; leaving out the two near-wall bins, a parabola
   fitted to the profile opens upward for A_SL = -35 (partially wetting:
   the liquid reaches further along the walls, contact angle below 90
   degrees), downward for A_SL = -20 (partially non-wetting, above 90
   degrees), its curvature falls from -35 over -30 to -20, and it is
   flattest at -30 (about 90 degrees).  Measured: relative curvatures
   +0.085, -0.048, -0.181.
"""
import numpy as np
import pytest

import oracle
from paper_1903_10134_amd import workloads as W
from test_gpu_parity import force_err, orc_params, pdiff, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mdpd():
    import torch
    assert torch.cuda.is_available()
    import paper_1903_10134_amd as m
    m.lib()
    return m


def test_slit_pore_parity_fp64(mdpd):
    w = W.slit_pore(A_SL=-35.0, seed=0)
    say("slit pore parity", w.n)
    s = mdpd.System(w, precision=mdpd.FP64)
    o = oracle.System(orc_params(w, search=1), w.x, w.v, w.types, w.frozen)
    for k in range(8):
        s.step(1)
        o.step(1)
        a, b = s.observables(), o.observables()
        assert a["ncorr_last"] == b["ncorr_last"], (k, a["ncorr_last"], b["ncorr_last"])
    st = o.state()
    x, v, rho = s.state()
    assert pdiff(x, st["x"], w.box) < 1e-10
    assert force_err(s.forces(), st["F"]) < 1e-10
    s.close()


def pore_profile(mdpd, A_SL, equil=4000, steps=10000, every=10, seed=0):
    """Time-averaged fluid count in the 8 bins of width r_c across the pore
    (y in [1, 9)), sampled every ``every`` steps after ``equil`` steps."""
    w = W.slit_pore(A_SL=A_SL, seed=seed)
    s = mdpd.System(w, precision=mdpd.FP32_FORCES)
    s.step(equil)
    acc = np.zeros(10)
    m = 0
    for _ in range(steps // every):
        s.step(every)
        acc += s.profile(1, 10, 0)
        m += 1
    ob = s.observables()
    s.close()
    counts = acc / m * (w.box[0] * 1.0 * w.box[2])  # number density x bin volume
    assert abs(counts.sum() - w.info["n_fluid"]) < 1e-6 * w.info["n_fluid"]
    return counts[1:9], ob


def curvature(counts):
    """Quadratic coefficient of a parabola through the six inner bins, in the
    pore coordinate eta in [-1, 1], relative to the mean count."""
    inner = counts[1:7]
    eta = (np.arange(8)[1:7] + 0.5 - 4.0) / 4.0
    c2 = np.polyfit(eta, inner, 2)[0]
    return float(c2 / inner.mean())


def test_contact_angle_trend(mdpd):
    res = {}
    for a in (-35.0, -30.0, -20.0):
        say("slit pore wetting", a)
        prof, ob = pore_profile(mdpd, a)
        res[a] = (prof, curvature(prof), ob)
    print()
    for a, (prof, c, ob) in res.items():
        print(f"A_SL {a:6.1f}: fluid per bin " + " ".join(f"{p:6.1f}" for p in prof) +
              f"  curvature {c:+.4f}  kT {ob['kT']:.3f}  corrections {ob['ncorr_total']}")
    c35, c30, c20 = res[-35.0][1], res[-30.0][1], res[-20.0][1]
    for a, (prof, c, ob) in res.items():
        assert prof.sum() > 0.97 * 4000, (a, prof.sum())  # the fluid stays in the pore
    assert c35 > 0.0 > c20
    assert c35 > c30 > c20
    assert abs(c30) < min(abs(c35), abs(c20))  # the flattest profile: about 90 degrees
