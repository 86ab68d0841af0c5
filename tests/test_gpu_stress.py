"""Pressure tensor on the GPU (needs an MI355X): parity with the oracle's
brute-force tensor, and the liquid-vacuum slab of Sec. 4.1 against the
values the paper prints for it.  Every case prints its name first.
"""
import json
import os

import numpy as np
import pytest

import oracle
from paper_1903_10134_amd import workloads as W
from test_gpu_parity import CASES, orc_params, say, small_channel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mdpd():
    import torch
    assert torch.cuda.is_available()
    import paper_1903_10134_amd as m
    m.lib()
    return m


@pytest.mark.parametrize("case", ["bulk_L10_n6000", "mixed_types", "dense_cluster", "small_channel"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_stress_matches_oracle(mdpd, case, prec):
    w = small_channel() if case == "small_channel" else CASES[case]
    say("stress", case, prec)
    s = mdpd.System(w, precision=mdpd.FP64 if prec == "fp64" else mdpd.FP32_FORCES)
    o = oracle.System(orc_params(w, search=1), w.x, w.v, w.types, w.frozen)
    s.step(2)
    o.step(2)
    P, Po = s.stress(), o.stress()
    scale = np.abs(Po[:3]).max()
    tol = 1e-12 if prec == "fp64" else 2e-5
    assert np.abs(P - Po).max() < tol * scale, (P, Po)
    # the FP32 form's scalar virial comes from the FP32 force pass, the tensor
    # from FP64 arithmetic on the same state
    rtol = 1e-9 if prec == "fp64" else 1e-5
    assert np.sum(P[:3]) / 3.0 == pytest.approx(s.observables()["pressure"], rel=rtol, abs=rtol * scale)
    s.close()


def fcc_slab(a=1.0, half=10, L=100.0, seed=0):
    """Face-centred cubic particles of lattice spacing a in a slab of
    thickness 2 half across x, filling y and z, centred in a periodic cube of
    edge L; Maxwell velocities at kT = 1."""
    basis = np.array([[0, 0, 0], [0.5, 0.5, 0], [0.5, 0, 0.5], [0, 0.5, 0.5]]) * a
    gx = np.arange(int(2 * half / a)) * a + (L / 2 - half)
    gy = np.arange(int(L / a)) * a
    cells = np.stack(np.meshgrid(gx, gy, gy, indexing="ij"), -1).reshape(-1, 3)
    x = (cells[:, None, :] + basis[None] + 0.25 * a).reshape(-1, 3)
    rng = np.random.default_rng(seed)
    v = rng.normal(size=x.shape)
    v -= v.mean(axis=0)
    return x, v


def test_liquid_vacuum_slab_density_and_tension(mdpd):
    """Sec. 4.1: a slab of mDPD water (A = -50, B = 25, r_d = 0.75, gamma =
    12.4) in a periodic 100^3 box, started from an fcc lattice with spacing
    r_c in |x| < 10, 5000 steps of equilibration, then 5000 steps of
    averaging.  The paper prints a density of 6.88 at the slab centre and an
    interfacial tension of 12.4 from the stress difference; the tension is
    checked here with L_x/2 (two interfaces) and printed with both factors."""
    import paper_1903_10134_amd as m
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "liquid_vacuum_slab.json")))
    x, v = fcc_slab()
    n = x.shape[0]
    say("liquid-vacuum slab", n)
    p = m.make_params(box=100.0, A=-50.0, B=25.0, gamma=12.4, rc=1.0, rd=0.75, kT=1.0, dt=0.01, seed=0,
                      precision=m.FP32_FORCES)
    s = m.System(params=p, x=x, v=v, types=np.zeros(n, np.int32), frozen=np.zeros(n, np.uint8))
    s.step(5000)
    prof, st = [], []
    for _ in range(100):
        s.step(50)
        prof.append(s.profile(0, 50, 0))
        st.append(s.stress())
    prof = np.mean(prof, axis=0)
    P = np.mean(st, axis=0)
    centre = 0.5 * (prof[24] + prof[25])  # bins [48, 50) and [50, 52)
    diff = P[0] - 0.5 * (P[1] + P[2])
    print(f"\nslab: centre density {centre:.3f} (paper 6.88); P_N - P_T = {diff:.4f}; "
          f"L_x/2 x that = {50.0 * diff:.2f}, L_x x that = {100.0 * diff:.2f} (paper 12.4)")
    s.close()
    assert abs(centre - gold["printed"]["centre_density"]) < 0.1
    assert abs(50.0 * diff - gold["printed"]["interfacial_tension"]) < 1.5
