"""Seeded synthetic inputs for the mDPD hot path.

This module only draws inputs (positions, velocities, particle types, frozen
wall masks, parameter tables); it holds none of the method's arithmetic.  It
is the one piece shared by the GPU tests, the benchmark and the oracle checks.

Workloads (all in DPD units, r_c = 1):

* ``bulk``      periodic cube at number density 6 with uniform-random
                positions and Maxwell velocities (mean removed, no rescale).
                L = 10 gives the 6,000-particle case, L = 56 the 1,053,696-
                particle case; this stands in for the per-GPU subdomain of
                about one million particles used in the paper's benchmarks.
* ``channel``   plane channel: fluid at density 6 in y in [0, Ly), frozen wall
                slabs of thickness 2 at density 6 on both sides (periodic box of
                height Ly + 4), body force along x.
* ``rock``      128^3 voxel mask from a seeded Gaussian random field
                (correlation length 6 voxels) thresholded to porosity 0.3; fluid
                at density 6 in pore voxels, frozen particles at density 6 in
                solid voxels within two voxels of a pore; deeper solid is left
                empty.  Stands in for the FIB-SEM shale pore images, which are
                not available.
* ``replicas``  independent periodic boxes with edges uniform in [8, 12],
                A ~ U[-50, -30], B ~ U[20, 30], one random stream per replica.
* ``ring_cells`` the manufactured homogeneous porous medium of Sec. 5.1 (the
                paper's scaling benchmark): 16 x 2 x 16 cells with a ring wall;
                23 x 23 cells (one layer) hold ~1.04M particles.
* ``slit_pore`` the static contact-angle set-up of Sec. 4.2: a 60 x 10 x 5
                box, 3,500 frozen particles in two wall layers of thickness
                r_c (y in [0, 1) and [9, 10), uniform random), 4,000 fluid
                particles uniform in x in [17, 43), y in [1, 9); two types
                (fluid 0, solid 1) with A_SS = A_LL = -40 and a chosen A_SL.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

# Parameters of the paper's mDPD fluid (Sec. 2.1, EOS figure): A = -40,
# B = 25, r_d = 0.75 r_c, gamma = 4.5, kT = 1; dt = 0.01 (Sec. 5.1).
MDPD_DEFAULTS = dict(A=-40.0, B=25.0, gamma=4.5, rc=1.0, rd=0.75, kT=1.0, dt=0.01, mass=1.0)


@dataclass
class Workload:
    name: str
    box: tuple
    x: np.ndarray          # (n, 3) float64
    v: np.ndarray          # (n, 3) float64
    types: np.ndarray      # (n,) int32
    frozen: np.ndarray     # (n,) uint8, 1 = frozen wall particle
    A: np.ndarray          # (T, T)
    B: np.ndarray
    gamma: np.ndarray
    rc: float = 1.0
    rd: float = 0.75
    kT: float = 1.0
    dt: float = 0.01
    mass: float = 1.0
    g: tuple = (0.0, 0.0, 0.0)
    seed: int = 0
    wall_model: int = 0
    phi_c: float = 0.5
    wall_slip: float = 0.0
    diss_ctrl: float = 0.0   # control of the effective fluid-solid dissipation (eta; 0: off)
    diss_rho: float = 0.0    # its fluid density rho_f
    info: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    def param_kwargs(self) -> dict:
        return dict(box=self.box, A=self.A, B=self.B, gamma=self.gamma, rc=self.rc, rd=self.rd,
                    kT=self.kT, dt=self.dt, mass=self.mass, g=self.g, seed=self.seed,
                    wall_model=self.wall_model, phi_c=self.phi_c, wall_slip=self.wall_slip,
                    diss_ctrl=self.diss_ctrl, diss_rho=self.diss_rho)


def _maxwell(rng, n, kT, mass, frozen):
    v = rng.normal(0.0, np.sqrt(kT / mass), size=(n, 3))
    v[frozen.astype(bool)] = 0.0
    fl = ~frozen.astype(bool)
    if fl.any():
        v[fl] -= v[fl].mean(axis=0)
    return v


def _table(val, T):
    return np.full((T, T), float(val))


def bulk(L=10.0, density=6.0, seed=0, A=-40.0, B=25.0, gamma=4.5, kT=1.0, dt=0.01, rd=0.75,
         n=None, box=None) -> Workload:
    """Uniform-random periodic fluid; n defaults to round(density * volume)."""
    box = tuple(float(b) for b in (box if box is not None else (L, L, L)))
    if n is None:
        n = int(round(density * box[0] * box[1] * box[2]))
    rng = np.random.Generator(np.random.PCG64(seed))
    x = rng.random((n, 3)) * np.asarray(box)
    frozen = np.zeros(n, np.uint8)
    v = _maxwell(rng, n, kT, 1.0, frozen)
    return Workload(name=f"bulk_L{box[0]:g}_n{n}", box=box, x=x, v=v,
                    types=np.zeros(n, np.int32), frozen=frozen, A=_table(A, 1), B=_table(B, 1),
                    gamma=_table(gamma, 1), kT=kT, dt=dt, rd=rd, seed=seed)


def channel(Lx=64.0, Ly=32.0, Lz=64.0, wall=2.0, density=6.0, seed=0, gx=0.02,
            A=-40.0, B=25.0, gamma=4.5, kT=1.0, dt=0.01) -> Workload:
    """Plane channel: fluid in y in [0, Ly), frozen slabs y in [-wall, 0) and
    [Ly, Ly + wall), stored in a periodic box of height Ly + 2*wall with the
    lower slab shifted to the top (y in [Ly + wall, Ly + 2 wall))."""
    rng = np.random.Generator(np.random.PCG64(seed))
    H = Ly + 2.0 * wall
    nf = int(round(density * Lx * Ly * Lz))
    nw = int(round(density * Lx * wall * Lz))
    xf = rng.random((nf, 3)) * np.array([Lx, Ly, Lz])
    w1 = rng.random((nw, 3)) * np.array([Lx, wall, Lz]) + np.array([0.0, Ly, 0.0])
    w2 = rng.random((nw, 3)) * np.array([Lx, wall, Lz]) + np.array([0.0, Ly + wall, 0.0])
    x = np.concatenate([xf, w1, w2])
    frozen = np.concatenate([np.zeros(nf, np.uint8), np.ones(2 * nw, np.uint8)])
    types = frozen.astype(np.int32)
    v = _maxwell(rng, x.shape[0], kT, 1.0, frozen)
    return Workload(name=f"channel_{Lx:g}x{Ly:g}x{Lz:g}", box=(Lx, H, Lz), x=x, v=v, types=types,
                    frozen=frozen, A=_table(A, 2), B=_table(B, 2), gamma=_table(gamma, 2), kT=kT,
                    dt=dt, g=(gx, 0.0, 0.0), seed=seed, wall_model=1,
                    info=dict(n_fluid=nf, n_wall=2 * nw, fluid_y=(0.0, Ly)))


def grf_mask(N=128, corr=6.0, porosity=0.3, seed=0):
    """Binary pore mask (True = pore) from white noise on a periodic N^3 grid
    smoothed by a Gaussian of standard deviation corr/sqrt(2) voxels (field
    autocorrelation exp(-r^2 / (2 corr^2))), thresholded at its porosity quantile."""
    rng = np.random.Generator(np.random.PCG64(seed))
    w = rng.standard_normal((N, N, N))
    k = np.fft.fftfreq(N) * 2.0 * np.pi
    kx, ky, kz = np.meshgrid(k, k, np.fft.rfftfreq(N) * 2.0 * np.pi, indexing="ij")
    s = corr / np.sqrt(2.0)
    filt = np.exp(-0.5 * s * s * (kx * kx + ky * ky + kz * kz))
    f = np.fft.irfftn(np.fft.rfftn(w) * filt, s=(N, N, N), axes=(0, 1, 2))
    thr = np.quantile(f, porosity)
    return f <= thr


def rock(N=128, corr=6.0, porosity=0.3, density=6.0, shell=2, seed=0, gx=0.01,
         A=-40.0, B=25.0, gamma=4.5, kT=1.0, dt=0.01) -> Workload:
    """Synthetic porous rock: fluid in pore voxels, frozen particles in solid
    voxels within ``shell`` voxels (periodic, 26-neighbour dilation) of a pore."""
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    pore = grf_mask(N, corr, porosity, seed)
    near = pore.copy()
    for _ in range(shell):
        grown = near.copy()
        for dx in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dz in (-1, 0, 1):
                    grown |= np.roll(near, (dx, dy, dz), axis=(0, 1, 2))
        near = grown
    wallvox = near & ~pore

    def fill(mask):
        idx = np.argwhere(mask).astype(np.float64)
        per = int(round(density))
        pts = np.repeat(idx, per, axis=0) + rng.random((idx.shape[0] * per, 3))
        return pts

    xf = fill(pore)
    xw = fill(wallvox)
    x = np.concatenate([xf, xw])
    nf, nw = xf.shape[0], xw.shape[0]
    frozen = np.concatenate([np.zeros(nf, np.uint8), np.ones(nw, np.uint8)])
    types = frozen.astype(np.int32)
    v = _maxwell(rng, x.shape[0], kT, 1.0, frozen)
    return Workload(name=f"rock_{N}", box=(float(N),) * 3, x=x, v=v, types=types, frozen=frozen,
                    A=_table(A, 2), B=_table(B, 2), gamma=_table(gamma, 2), kT=kT, dt=dt,
                    g=(gx, 0.0, 0.0), seed=seed, wall_model=1,
                    info=dict(n_fluid=nf, n_wall=nw, porosity=float(pore.mean())))


def replicas(count=256, lo=8.0, hi=12.0, density=6.0, seed=0, kT=1.0, dt=0.01, gamma=4.5):
    """Independent periodic boxes with edge ~U[lo, hi], A ~ U[-50,-30],
    B ~ U[20,30]; replica r draws from its own stream spawned from ``seed``."""
    ss = np.random.SeedSequence(seed)
    out = []
    for r, child in enumerate(ss.spawn(count)):
        rng = np.random.Generator(np.random.PCG64(child))
        L = float(rng.uniform(lo, hi))
        A = float(rng.uniform(-50.0, -30.0))
        B = float(rng.uniform(20.0, 30.0))
        n = int(round(density * L ** 3))
        x = rng.random((n, 3)) * L
        frozen = np.zeros(n, np.uint8)
        v = _maxwell(rng, n, kT, 1.0, frozen)
        out.append(Workload(name=f"replica{r}", box=(L, L, L), x=x, v=v,
                            types=np.zeros(n, np.int32), frozen=frozen, A=_table(A, 1),
                            B=_table(B, 1), gamma=_table(gamma, 1), kT=kT, dt=dt,
                            seed=(seed * 7919 + r) & 0xFFFFFFFF))
    return out


def lattice_sc(ncell_per_edge=6, density=6.0):
    """Simple-cubic lattice at the given number density (spacing density^-1/3)."""
    a = density ** (-1.0 / 3.0)
    m = int(ncell_per_edge)
    g = np.arange(m) * a
    x = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3) + 0.5 * a
    return x, m * a


def lattice_fcc(m=4, a=1.0):
    """Face-centred cubic lattice of m^3 conventional cells of edge a."""
    basis = np.array([[0, 0, 0], [0.5, 0.5, 0], [0.5, 0, 0.5], [0, 0.5, 0.5]]) * a
    g = np.arange(m) * a
    cells = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    x = (cells[:, None, :] + basis[None, :, :]).reshape(-1, 3) + 0.25 * a
    return x, m * a


def slit_pore(A_SL=-35.0, seed=0, n_solid=3500, n_fluid=4000, B=25.0, gamma=4.5, kT=1.0, dt=0.01):
    """Sec. 4.2 slit nano channel: the paper's domain x in [-30, 30],
    y in [-5, 5], z in [-2.5, 2.5] shifted to [0, 60) x [0, 10) x [0, 5).
    Solid particles fill y in [0, 1) and [9, 10) (half each; the two layers
    meet across the periodic y boundary), fluid starts in x in [17, 43),
    y in [1, 9).  Types: fluid 0, solid 1; A_SS = A_LL = -40, A_SL varies,
    B = 25 for every pair, r_d = 0.75.  Walls use the boundary-volume-
    fraction model."""
    rng = np.random.Generator(np.random.PCG64(seed))
    box = (60.0, 10.0, 5.0)
    h = n_solid // 2
    lo = rng.random((h, 3)) * np.array([60.0, 1.0, 5.0])
    hi = rng.random((n_solid - h, 3)) * np.array([60.0, 1.0, 5.0]) + np.array([0.0, 9.0, 0.0])
    xf = rng.random((n_fluid, 3)) * np.array([26.0, 8.0, 5.0]) + np.array([17.0, 1.0, 0.0])
    x = np.concatenate([xf, lo, hi])
    frozen = np.concatenate([np.zeros(n_fluid, np.uint8), np.ones(n_solid, np.uint8)])
    types = frozen.astype(np.int32)
    v = _maxwell(rng, x.shape[0], kT, 1.0, frozen)
    A = np.array([[-40.0, A_SL], [A_SL, -40.0]])
    return Workload(name=f"slit_pore_ASL{A_SL:g}", box=box, x=x, v=v, types=types, frozen=frozen, A=A,
                    B=_table(B, 2), gamma=_table(gamma, 2), kT=kT, dt=dt, seed=seed, wall_model=1,
                    info=dict(n_fluid=n_fluid, n_wall=n_solid, pore_y=(1.0, 9.0)))


def ring_cells(n=23, layers=1, seed=0, solid_density=8.0, fluid_density=6.2, gz=0.02, B=25.0, gamma=4.5,
               kT=1.0, dt=0.01):
    """Sec. 5.1 manufactured homogeneous porous medium: square cells of
    16 x 2 x 16 (x, y, z), each with a ring-shaped solid wall (outer radius 7,
    inner radius 6, axis along y) at number density 8 and fluid at density 6.2
    outside the ring; n x n cells in the x-z plane, the cells of every other
    row (in z) shifted by half a cell in x; periodic in all directions, body
    force g_z on the fluid.  The paper's cell is 2 thick in y (one layer);
    ``layers`` copies of it can be stacked along y.  23 x 23 cells of one
    layer (about 1.04 M particles) are the per-GPU size of the paper's weak
    scaling runs.  Particles are placed uniformly at random in
    their regions (the paper equilibrates them first).  Types: fluid 0, solid
    1, A = -40 between all pairs, B = 25, r_d = 0.75."""
    rng = np.random.Generator(np.random.PCG64(seed))
    C, H = 16.0, 2.0 * layers
    box = (C * n, H, C * n)
    r_out, r_in = 7.0, 6.0
    ring_area = np.pi * (r_out ** 2 - r_in ** 2)
    fluid_area = C * C - np.pi * r_out ** 2
    n_solid = int(round(solid_density * ring_area * H))
    n_fluid = int(round(fluid_density * fluid_area * H))

    def ring(count):
        # uniform in the annulus: radius from the area-weighted distribution
        rad = np.sqrt(rng.uniform(r_in ** 2, r_out ** 2, count))
        ang = rng.uniform(0.0, 2.0 * np.pi, count)
        return np.stack([C / 2 + rad * np.cos(ang), rng.uniform(0.0, H, count), C / 2 + rad * np.sin(ang)], 1)

    def outside(count):
        pts = np.empty((0, 3))
        while pts.shape[0] < count:
            p = rng.random((2 * count, 3)) * np.array([C, H, C])
            keep = (p[:, 0] - C / 2) ** 2 + (p[:, 2] - C / 2) ** 2 >= r_out ** 2
            pts = np.concatenate([pts, p[keep]])
        return pts[:count]

    xs, xf = [], []
    for iz in range(n):
        for ix in range(n):
            off = np.array([C * ix + (C / 2 if iz % 2 == 1 else 0.0), 0.0, C * iz])
            xs.append(ring(n_solid) + off)
            xf.append(outside(n_fluid) + off)
    xf = np.concatenate(xf)
    xs = np.concatenate(xs)
    x = np.concatenate([xf, xs])
    x[:, 0] %= box[0]
    frozen = np.concatenate([np.zeros(xf.shape[0], np.uint8), np.ones(xs.shape[0], np.uint8)])
    types = frozen.astype(np.int32)
    v = _maxwell(rng, x.shape[0], kT, 1.0, frozen)
    return Workload(name=f"ring_cells_{n}x{n}", box=box, x=x, v=v, types=types, frozen=frozen,
                    A=_table(-40.0, 2), B=_table(B, 2), gamma=_table(gamma, 2), kT=kT, dt=dt,
                    g=(0.0, 0.0, gz), seed=seed, wall_model=1,
                    info=dict(n_fluid=int(xf.shape[0]), n_wall=int(xs.shape[0]), cells=n * n,
                              per_cell=(n_solid, n_fluid)))
