"""Walled-step parity on irregular voxel pore geometries (Sec. 2.2, 2.3) against
the FP64 oracle (needs an MI355X).

The pore space is a small periodic Gaussian-random-field mask; its surface
wall voxels are filled with frozen particles either by the lattice-like
packing or by patches of a database that the oracle itself equilibrated
(no input of these tests comes from the GPU path).  The GPU steps the system
beside the oracle: the boundary-volume-fraction corrector must reject the
same number of predicted moves at every step, and in the FP64 form forces
and positions stay within 1e-10 over the whole run.
"""
import numpy as np
import pytest

import oracle
from paper_1903_10134_amd import packing as K
from paper_1903_10134_amd import workloads as W
from test_gpu_parity import FP32_TOL, force_err, orc_params, pdiff, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mdpd():
    import torch
    assert torch.cuda.is_available()
    import paper_1903_10134_amd as m
    m.lib()
    return m


def oracle_patch_db(boxes=4, edge=4, density=8.0, steps=200, seed=11):
    """Patch database equilibrated by the oracle: periodic cubes of edge 4 at
    the solid density, uniform-random start, `steps` FP64 steps, cut into
    unit voxels."""
    cuts = []
    for r in range(boxes):
        L = float(edge)
        w = W.bulk(L=L, density=density, seed=seed + r)
        o = oracle.System(orc_params(w, search=1), w.x, w.v)
        o.step(steps)
        cuts.append(K.cut_patches(o.state()["x"], (L, L, L), 1.0))
    return K.merge_patches(cuts)


@pytest.fixture(scope="module")
def db():
    return oracle_patch_db()


def pore_mask():
    pore = W.grf_mask(16, corr=3.0, porosity=0.4, seed=4)
    assert 0.3 < pore.mean() < 0.5
    return pore


@pytest.mark.parametrize("wall", ["patch", "lattice"])
def test_voxel_walls_fp64_parity(mdpd, db, wall):
    w = K.voxel_workload(pore_mask(), h=1.0, fluid_density=6.0, wall=wall, db=db, seed=6,
                         g=(0.05, 0.0, 0.0))
    say("voxel walls fp64", wall, w.n, w.info["n_wall"])
    s = mdpd.System(w, precision=mdpd.FP64)
    o = oracle.System(orc_params(w, search=1), w.x, w.v, w.types, w.frozen)
    total = 0
    for k in range(12):
        s.step(1)
        o.step(1)
        a, b = s.observables(), o.observables()
        assert a["ncorr_last"] == b["ncorr_last"], (k, a["ncorr_last"], b["ncorr_last"])
        total += b["ncorr_last"]
        st = o.state()
        x, v, rho = s.state()
        assert pdiff(x, st["x"], w.box) < 1e-10, k
        assert np.abs(v - st["v"]).max() < 1e-10, k
        assert force_err(s.forces(), st["F"]) < 1e-10, k
    assert total > 0, "the case should exercise the corrector"
    print(f"\n{wall}: {w.n} particles ({w.info['n_wall']} frozen), {total} corrections in 12 steps")
    s.close()


def test_voxel_walls_fp32_first_steps(mdpd, db):
    """FP32 pair forces: the same corrector decisions and forces within the
    FP32 bar over the first steps."""
    w = K.voxel_workload(pore_mask(), h=1.0, fluid_density=6.0, wall="patch", db=db, seed=6,
                         g=(0.05, 0.0, 0.0))
    say("voxel walls fp32", w.n)
    s = mdpd.System(w, precision=mdpd.FP32_FORCES)
    o = oracle.System(orc_params(w, search=1), w.x, w.v, w.types, w.frozen)
    for k in range(3):
        s.step(1)
        o.step(1)
        assert s.observables()["ncorr_last"] == o.observables()["ncorr_last"], k
        assert force_err(s.forces(), o.state()["F"]) < 10 * FP32_TOL * (k + 1), k
    s.close()
