"""Pore-surface walls from voxel data (Sec. 2.3).

A porous sample is a periodic grid of voxels of edge h, each pore or solid.
Building its walls takes two sweeps:

1. ``surface_wall_voxels``: the solid voxels within a Chebyshev distance of
   t = ceil(r_c / h) voxels of a pore voxel.  Every solid point closer than
   r_c to the pore space lies in such a voxel, so a fluid particle always
   sees a wall at least r_c thick; deeper solid stays empty.
2. Filling them with frozen particles at the solid number density:
   * ``fill_lattice``: the earlier lattice-like packing, the same simple-cubic
     arrangement in every voxel;
   * ``fill_patches``: the improved insertion, where each voxel gets a locally
     equilibrated particle patch drawn at random from a database prepared in
     advance (``build_patch_database``: periodic boxes of the solid
     equilibrated with the mDPD step on the GPU, cut into voxel-sized cubes
     by ``cut_patches``), in one of the 48 symmetries of the cube.

``voxel_workload`` assembles a walled system from a pore mask: fluid at its
density in the pore voxels (uniform random), frozen wall particles from one
of the fills, two types, boundary-volume-fraction walls.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass

import numpy as np

from .workloads import MDPD_DEFAULTS, Workload, _maxwell, _table


def surface_wall_voxels(pore: np.ndarray, t: int) -> np.ndarray:
    """Solid voxels (``~pore``) within Chebyshev distance ``t`` (in voxels,
    periodic) of a pore voxel: a dilation of the pore mask by a cube of
    half-width t, one axis at a time."""
    if t < 0:
        raise ValueError("t must be >= 0")
    near = np.asarray(pore, bool).copy()
    for ax in range(3):
        grown = near.copy()
        for d in range(1, t + 1):
            grown |= np.roll(near, d, axis=ax)
            grown |= np.roll(near, -d, axis=ax)
        near = grown
    return near & ~np.asarray(pore, bool)


def wall_thickness_voxels(h: float, rc: float = 1.0) -> int:
    """t = ceil(r_c / h): the voxel reach that covers a wall of thickness r_c."""
    return int(np.ceil(rc / h - 1e-12))


def lattice_patch(h: float, density: float) -> np.ndarray:
    """The lattice-like voxel filling: m^3 points of a simple-cubic lattice of
    spacing h / m at the cell centres, m = round((density h^3)^(1/3))."""
    m = max(1, int(round((density * h ** 3) ** (1.0 / 3.0))))
    g = (np.arange(m) + 0.5) * (h / m)
    return np.array(list(itertools.product(g, g, g)), dtype=np.float64)


def fill_lattice(surface: np.ndarray, h: float, density: float) -> np.ndarray:
    """Frozen positions of the lattice-like packing of every surface voxel."""
    pat = lattice_patch(h, density)
    idx = np.argwhere(surface).astype(np.float64) * h
    return (idx[:, None, :] + pat[None, :, :]).reshape(-1, 3)


@dataclass
class PatchDB:
    """Voxel patches: patch k holds pos[off[k]:off[k+1]], coordinates
    relative to the voxel's lower corner, in [0, h)."""
    h: float
    pos: np.ndarray   # (M, 3) float64
    off: np.ndarray   # (K + 1,) int64

    @property
    def count(self) -> int:
        return int(self.off.shape[0] - 1)

    def patch(self, k: int) -> np.ndarray:
        return self.pos[self.off[k]:self.off[k + 1]]


def cut_patches(x: np.ndarray, box, h: float) -> PatchDB:
    """Cuts a periodic box whose edges are whole multiples of h into its
    voxel-sized cubes: every particle lands in exactly one patch."""
    box = np.asarray(box, np.float64)
    nv = np.rint(box / h).astype(np.int64)
    if np.any(np.abs(nv * h - box) > 1e-9 * box) or np.any(nv < 1):
        raise ValueError("box edges must be whole multiples of h")
    xw = np.mod(np.asarray(x, np.float64), box)
    c = np.minimum(np.floor(xw / h).astype(np.int64), nv - 1)
    key = c[:, 0] + nv[0] * (c[:, 1] + nv[1] * c[:, 2])
    order = np.argsort(key, kind="stable")
    rel = xw[order] - c[order] * h
    rel = np.clip(rel, 0.0, np.nextafter(h, 0.0))
    counts = np.bincount(key, minlength=int(nv.prod()))
    off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    return PatchDB(h=h, pos=rel, off=off)


def merge_patches(dbs) -> PatchDB:
    dbs = list(dbs)
    if not dbs:
        raise ValueError("no patch databases to merge")
    h = dbs[0].h
    pos = np.concatenate([d.pos for d in dbs])
    counts = np.concatenate([np.diff(d.off) for d in dbs])
    return PatchDB(h=h, pos=pos, off=np.concatenate([[0], np.cumsum(counts)]).astype(np.int64))


# The 48 symmetries of the cube [0, h)^3: an axis permutation, then a
# reflection x -> h - x on any subset of the axes.
CUBE_SYMMETRIES = [(p, f) for p in itertools.permutations(range(3)) for f in itertools.product((0, 1), repeat=3)]


def apply_symmetry(p: np.ndarray, h: float, sym) -> np.ndarray:
    perm, flip = sym
    q = p[:, list(perm)].copy()
    for a in range(3):
        if flip[a]:
            q[:, a] = h - q[:, a]
    # h - x maps [0, h) onto (0, h]; keep the patch inside its voxel
    return np.clip(q, 0.0, np.nextafter(h, 0.0))


def fill_patches(surface: np.ndarray, db: PatchDB, seed: int = 0, symmetries: bool = True):
    """Frozen positions of the patch packing: every surface voxel takes patch
    k ~ U{0..K-1} (and a symmetry ~ U{0..47}) from its own draw of the seeded
    stream; the output lists the voxels in ``argwhere`` order, each with its
    patch's particles in database order.  Returns (positions, patch index per
    voxel)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    vox = np.argwhere(surface)
    pick = rng.integers(0, db.count, size=vox.shape[0])
    syms = rng.integers(0, len(CUBE_SYMMETRIES), size=vox.shape[0]) if symmetries else \
        np.zeros(vox.shape[0], np.int64)
    counts = np.diff(db.off)[pick]
    total = int(counts.sum())
    if total == 0:
        return np.zeros((0, 3)), pick
    # source row of every output particle: patch start + rank inside the patch
    first = np.cumsum(counts) - counts
    src = np.repeat(db.off[pick], counts) + (np.arange(total) - np.repeat(first, counts))
    owner = np.repeat(np.arange(vox.shape[0]), counts)
    sym_of = syms[owner]
    x = np.empty((total, 3))
    for k in np.unique(sym_of):
        sel = sym_of == k
        p = db.pos[src[sel]]
        x[sel] = apply_symmetry(p, db.h, CUBE_SYMMETRIES[int(k)]) if symmetries else p
    x += vox[owner] * db.h
    return x, pick


def build_patch_database(boxes: int = 8, edge_voxels: int = 4, h: float = 1.0, density: float = 8.0,
                         steps: int = 500, seed: int = 0, precision=None, **mdpd) -> PatchDB:
    """The database of locally equilibrated patches: ``boxes`` periodic cubes
    of edge_voxels * h at the solid density, uniform-random start, advanced
    ``steps`` mDPD steps as one batch on the GPU (parameters of the solid
    from ``mdpd``, the paper's fluid by default), then cut into voxels:
    boxes * edge_voxels^3 patches."""
    from . import _native as nat
    prm = dict(MDPD_DEFAULTS)
    prm.update(mdpd)
    L = edge_voxels * h
    if L < 3.0 * prm["rc"]:
        raise ValueError("the equilibration box needs at least 3 r_c per edge")
    ss = np.random.SeedSequence(seed)
    reps = []
    for r, child in enumerate(ss.spawn(boxes)):
        rng = np.random.Generator(np.random.PCG64(child))
        n = int(round(density * L ** 3))
        x = rng.random((n, 3)) * L
        frozen = np.zeros(n, np.uint8)
        v = _maxwell(rng, n, prm["kT"], prm["mass"], frozen)
        reps.append(Workload(name=f"patchbox{r}", box=(L, L, L), x=x, v=v, types=np.zeros(n, np.int32),
                             frozen=frozen, A=_table(prm["A"], 1), B=_table(prm["B"], 1),
                             gamma=_table(prm["gamma"], 1), rc=prm["rc"], rd=prm["rd"], kT=prm["kT"],
                             dt=prm["dt"], mass=prm["mass"], seed=(seed * 104729 + r) & 0xFFFFFFFF))
    b = nat.Batch(reps, precision=nat.FP32_FORCES if precision is None else precision)
    try:
        b.step(steps)
        x, _, _ = b.state(with_rho=False)
    finally:
        b.close()
    off = np.concatenate([[0], np.cumsum([r.n for r in reps])])
    return merge_patches(cut_patches(x[off[r]:off[r + 1]], (L, L, L), h) for r in range(boxes))


def voxel_workload(pore: np.ndarray, h: float = 1.0, fluid_density: float = 6.0, wall: str = "patch",
                   db: PatchDB | None = None, solid_density: float = 8.0, seed: int = 0,
                   g=(0.0, 0.0, 0.0), A=-40.0, A_SL=None, B=25.0, gamma=4.5, kT=1.0, dt=0.01,
                   rc: float = 1.0, rd: float = 0.75) -> Workload:
    """A walled system from a periodic pore mask (True = pore) of voxel edge
    h: fluid uniform at ``fluid_density`` in the pore voxels (type 0), frozen
    wall particles in the surface wall voxels (type 1) from the lattice
    (``wall="lattice"``) or patch (``wall="patch"``, needs ``db``) packing."""
    pore = np.asarray(pore, bool)
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    surface = surface_wall_voxels(pore, wall_thickness_voxels(h, rc))
    if wall == "lattice":
        xw = fill_lattice(surface, h, solid_density)
    elif wall == "patch":
        if db is None:
            raise ValueError("the patch packing needs a patch database")
        if abs(db.h - h) > 1e-12:
            raise ValueError("the database was cut for another voxel edge")
        xw, _ = fill_patches(surface, db, seed=seed + 2)
    else:
        raise ValueError(f"unknown wall packing {wall!r}")
    pv = np.argwhere(pore).astype(np.float64)
    per = fluid_density * h ** 3
    counts = rng.poisson(per, size=pv.shape[0]) if abs(per - round(per)) > 1e-12 else \
        np.full(pv.shape[0], int(round(per)))
    xf = (np.repeat(pv, counts, axis=0) + rng.random((int(counts.sum()), 3))) * h
    x = np.concatenate([xf, xw])
    nf, nw = xf.shape[0], xw.shape[0]
    frozen = np.concatenate([np.zeros(nf, np.uint8), np.ones(nw, np.uint8)])
    types = frozen.astype(np.int32)
    v = _maxwell(rng, x.shape[0], kT, 1.0, frozen)
    Atab = _table(A, 2)
    if A_SL is not None:
        Atab[0, 1] = Atab[1, 0] = A_SL
    box = tuple(float(s * h) for s in pore.shape)
    return Workload(name=f"voxel_{wall}", box=box, x=x, v=v, types=types, frozen=frozen, A=Atab,
                    B=_table(B, 2), gamma=_table(gamma, 2), rc=rc, rd=rd, kT=kT, dt=dt, g=tuple(g),
                    seed=seed, wall_model=1,
                    info=dict(n_fluid=nf, n_wall=nw, surface_voxels=int(surface.sum()),
                              porosity=float(pore.mean())))
