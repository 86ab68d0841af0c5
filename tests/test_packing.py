"""Pore-surface wall packing from voxels (Sec. 2.3), host part: the surface
voxel sweep, the lattice and patch fills, the database cut.  Brute force on
small grids and invariants (every particle lands in one patch, cube
symmetries keep a patch's pair distances, every solid point within r_c of the
pore space is covered)."""
import itertools

import numpy as np
import pytest

from paper_1903_10134_amd import packing as K


def brute_surface(pore, t):
    """Solid voxels with a pore voxel at periodic Chebyshev distance <= t."""
    shp = np.array(pore.shape)
    pv = np.argwhere(pore)
    out = np.zeros_like(pore)
    for v in np.argwhere(~pore):
        d = np.abs(pv - v)
        d = np.minimum(d, shp - d)
        out[tuple(v)] = bool(len(pv)) and bool(np.any(d.max(axis=1) <= t))
    return out


@pytest.mark.parametrize("t", [0, 1, 2])
@pytest.mark.parametrize("seed", [0, 1])
def test_surface_voxels_match_brute_force(t, seed):
    rng = np.random.default_rng(seed)
    pore = rng.random((7, 6, 5)) < 0.2
    got = K.surface_wall_voxels(pore, t)
    assert np.array_equal(got, brute_surface(pore, t))
    assert not np.any(got & pore)


def test_thickness_in_voxels():
    assert K.wall_thickness_voxels(1.0) == 1
    assert K.wall_thickness_voxels(0.5) == 2
    assert K.wall_thickness_voxels(0.4) == 3
    assert K.wall_thickness_voxels(1.0 / 3.0) == 3
    assert K.wall_thickness_voxels(2.0) == 1


def test_solid_within_rc_of_pore_is_covered():
    """Random points in solid voxels: those closer than r_c to the pore
    space (distance to the nearest pore voxel's box, periodic) lie in surface
    voxels, for voxel edges 1 and 0.5."""
    rng = np.random.default_rng(3)
    for h in (1.0, 0.5):
        pore = rng.random((10, 9, 8)) < 0.15
        surf = K.surface_wall_voxels(pore, K.wall_thickness_voxels(h, 1.0))
        box = np.array(pore.shape) * h
        pv = np.argwhere(pore) * h
        solid = np.argwhere(~pore)
        pts = (solid[rng.integers(0, len(solid), 3000)] + rng.random((3000, 3))) * h
        covered = checked = 0
        for p in pts:
            lo = pv - p
            lo = lo - box * np.rint(lo / box)
            gap = np.maximum(0.0, np.maximum(lo, -(lo + h)))   # per-axis gap to the voxel [c, c + h)
            dist = np.sqrt((gap ** 2).sum(axis=1)).min()
            if dist < 1.0:
                checked += 1
                covered += surf[tuple(np.floor(p / h).astype(int))]
        assert checked > 100 and covered == checked


def test_lattice_fill():
    p = K.lattice_patch(1.0, 8.0)
    assert p.shape == (8, 3)
    assert np.array_equal(np.unique(p), [0.25, 0.75])
    assert K.lattice_patch(0.5, 8.0).shape == (1, 3)
    surf = np.zeros((4, 5, 6), bool)
    surf[1, 2, 3] = surf[0, 0, 0] = True
    x = K.fill_lattice(surf, 1.0, 8.0)
    assert x.shape == (16, 3)
    cells = {tuple(c) for c in np.floor(x).astype(int)}
    assert cells == {(1, 2, 3), (0, 0, 0)}


def test_cut_patches_partitions_the_box():
    rng = np.random.default_rng(5)
    L = 4.0
    x = rng.random((512, 3)) * L
    x[0] = [L - 1e-17, 0.0, 3.9999999999999996]     # at the upper edges
    db = K.cut_patches(x, (L, L, L), 1.0)
    assert db.count == 64 and db.off[-1] == 512
    assert np.all(db.pos >= 0.0) and np.all(db.pos < 1.0)
    # put every patch back at its voxel: the same multiset of positions
    back = []
    for k in range(db.count):
        c = np.array([k % 4, (k // 4) % 4, k // 16], np.float64)
        back.append(db.patch(k) + c)
    back = np.concatenate(back)
    a = np.sort(np.round(np.mod(x, L), 12).view([("", float)] * 3).ravel())
    b = np.sort(np.round(back, 12).view([("", float)] * 3).ravel())
    assert np.array_equal(a, b)
    with pytest.raises(ValueError):
        K.cut_patches(x, (4.5, 4.0, 4.0), 1.0)


def test_cube_symmetries():
    syms = K.CUBE_SYMMETRIES
    assert len(syms) == 48
    rng = np.random.default_rng(7)
    p = rng.random((9, 3)) * 0.5
    d0 = np.linalg.norm(p[:, None] - p[None], axis=2)
    images = set()
    for s in syms:
        q = K.apply_symmetry(p, 0.5, s)
        assert np.all(q >= 0.0) and np.all(q < 0.5)
        assert np.allclose(np.linalg.norm(q[:, None] - q[None], axis=2), d0, atol=1e-14)
        images.add(tuple(np.round(q, 12).ravel()))
    assert len(images) == 48        # a generic patch has 48 distinct images


def test_fill_patches():
    rng = np.random.default_rng(9)
    db = K.cut_patches(rng.random((8 * 27, 3)) * 3.0, (3.0, 3.0, 3.0), 1.0)
    surf = rng.random((5, 4, 6)) < 0.3
    x, pick = K.fill_patches(surf, db, seed=4)
    vox = np.argwhere(surf)
    assert len(pick) == len(vox)
    counts = np.diff(db.off)[pick]
    assert x.shape[0] == counts.sum()
    # each voxel's particles sit inside it, as many as its patch holds
    cell = np.floor(x).astype(int)
    start = 0
    for v, c in zip(vox, counts):
        assert np.all(cell[start:start + c] == v)
        start += c
    x2, pick2 = K.fill_patches(surf, db, seed=4)
    assert np.array_equal(x, x2) and np.array_equal(pick, pick2)


def test_voxel_workload_slab():
    pore = np.zeros((6, 8, 4), bool)
    pore[:, 2:6, :] = True
    w = K.voxel_workload(pore, h=1.0, fluid_density=6.0, wall="lattice", seed=1, g=(0.02, 0, 0))
    nf, nw = w.info["n_fluid"], w.info["n_wall"]
    assert nf == 6 * 4 * 4 * 6 and nw == 2 * 6 * 4 * 8
    assert w.box == (6.0, 8.0, 4.0) and w.wall_model == 1
    yf, yw = w.x[:nf, 1], w.x[nf:, 1]
    assert np.all((yf >= 2.0) & (yf < 6.0))
    assert np.all(((yw >= 1.0) & (yw < 2.0)) | ((yw >= 6.0) & (yw < 7.0)))
    assert np.array_equal(w.frozen, np.r_[np.zeros(nf), np.ones(nw)].astype(np.uint8))
    assert np.all(w.v[nf:] == 0.0)
    with pytest.raises(ValueError):
        K.voxel_workload(pore, wall="patch")
