"""The synthetic rock at its full size and length (needs an MI355X).

Config: a 128^3-voxel Gaussian-random-field mask (correlation length 6
voxels) at porosity 0.3, one DPD unit per voxel, frozen particles at density
6 in the two voxel layers of solid around the pores (the deeper solid is
empty), fluid at density 6 in the pores (7,574,448 particles, 3,774,876 of
them fluid), body force g_x = 0.01, boundary-volume-fraction walls with
bounce-back, FP32 forces, 2,000 steps from the uniform-random filling.

The filling starts hot (random overlaps: kT 1.3 after 100 steps); the test
shows that the walled step settles: kT within 1% of the set value from step
500 on, the wall corrections per step level off instead of growing, the
fluid flows along the force, and no fluid particle ever reaches the empty
solid beyond the wall layers.
"""
import numpy as np
import pytest

from paper_1903_10134_amd import packing as K
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


def test_rock_settles_over_2000_steps(mdpd):
    w = W.rock()
    say("rock 128^3", w.n)
    nf = int(w.n - int(np.asarray(w.frozen).sum()))
    # the voxels a fluid particle may occupy: pores and the two wall layers
    pore = W.grf_mask(128, 6.0, 0.3, 0)
    allowed = pore | K.surface_wall_voxels(pore, 2)
    s = mdpd.System(w, precision=mdpd.FP32_FORCES)
    kt, corr, vx = [], [], []
    c0 = 0
    for _ in range(20):
        s.step(100)
        o = s.observables()
        kt.append(o["kT"])
        corr.append((o["ncorr_total"] - c0) / 100.0)
        c0 = o["ncorr_total"]
        vx.append(o["momentum"][0] / nf)
    x, _, _ = s.state()
    s.close()
    c = np.floor(x[:nf]).astype(int) % 128
    leaked = int((~allowed[c[:, 0], c[:, 1], c[:, 2]]).sum())
    late = np.asarray(vx[10:])
    print(f"\nrock: kT every 100 steps {' '.join(f'{t:.4f}' for t in kt)}")
    print(f"rock: corrections per step {' '.join(f'{v:.0f}' for v in corr)}")
    print(f"rock: mean fluid v_x over steps 1100..2000 {late.mean():.5f} +- "
          f"{late.std(ddof=1) / np.sqrt(len(late)):.5f}; fluid beyond the wall layers {leaked}")
    assert np.all(np.abs(np.asarray(kt[4:]) - 1.0) < 0.01), kt
    assert max(corr[10:]) <= corr[4], corr
    assert late.mean() > 3.0 * late.std(ddof=1) / np.sqrt(len(late)), late
    assert leaked == 0
