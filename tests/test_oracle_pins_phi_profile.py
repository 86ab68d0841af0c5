"""Pins of two oracle functions that every wall and profile parity claim
rests on: the boundary volume fraction phi (Sec. 2.2, wall reading) and the
bin profiles (Sec. 4.1 density profile, Sec. 4.2 / 5 flow profiles).

Each case has a closed form that a plausible mistake breaks, and the test
states the value such a mistake would give, so a change of the weight (w_c
for w_c^2), of the cutoff of a sum (r_d for r_c), of the bin index, of the
bin volume or of the mean subtraction of the temperature fails here.  CPU
only.
"""
import numpy as np
import pytest

RC, RD, L = 1.0, 0.75, 10.0


def wc(r):
    return max(0.0, 1.0 - r / RC)


def params(orc, box=L, **kw):
    return orc.make_params(box=box, A=-40.0, B=25.0, gamma=4.5, rc=RC, rd=RD, wall_model=1, **kw)


# --------------------------------------------------------------------------
# Boundary volume fraction
# --------------------------------------------------------------------------
@pytest.mark.parametrize("search", [0, 1])
def test_phi_of_three_particles(orc, search):
    """Fluid i at the origin, frozen a at r1 = 0.3 on x, fluid b at r2 = 0.8
    on y (beyond r_d, inside r_c); |a - b| = sqrt(0.73) < r_c.
      phi_i = w(r1)^2 / (w(r1)^2 + w(r2)^2)        = 0.924528...
      phi_b = w(r_ab)^2 / (w(r_ab)^2 + w(r2)^2)
    A plain w weight would give 0.636 / 0.9245 -> 0.875 for phi_i; a
    denominator cut at r_d would give 1.0; frozen particles get 0."""
    p = params(orc, search=search)
    c = np.array([5.0, 5.0, 5.0])
    x = np.array([c, c + [0.3, 0.0, 0.0], c + [0.0, 0.8, 0.0]])
    fz = np.array([0, 1, 0], np.uint8)
    phi = orc.phi(p, x, fz)
    rab = np.sqrt(0.3**2 + 0.8**2)
    exp_i = wc(0.3) ** 2 / (wc(0.3) ** 2 + wc(0.8) ** 2)
    exp_b = wc(rab) ** 2 / (wc(rab) ** 2 + wc(0.8) ** 2)
    assert phi[0] == pytest.approx(exp_i, rel=1e-14)
    assert phi[2] == pytest.approx(exp_b, rel=1e-14)
    assert phi[1] == 0.0
    # what the mutations would give: each is far outside the tolerance
    assert abs(phi[0] - wc(0.3) / (wc(0.3) + wc(0.8))) > 0.05
    assert abs(phi[0] - 1.0) > 0.05


def test_phi_counts_only_neighbours_within_rc_and_across_the_boundary(orc):
    """The frozen neighbour sits across the periodic boundary (x = 0.1 and
    x = L - 0.2: distance 0.3); a second frozen particle at exactly r_c is not
    a neighbour (strict cutoff), and a fluid one at 1.2 is not either.  A
    lone fluid particle has phi = 0 (empty sums)."""
    p = params(orc)
    x = np.array([[0.1, 5.0, 5.0], [L - 0.2, 5.0, 5.0], [0.1, 6.0, 5.0], [0.1, 5.0, 6.2],
                  [0.1, 5.5, 5.0], [7.0, 2.0, 2.0]])
    fz = np.array([0, 1, 1, 0, 0, 0], np.uint8)
    phi = orc.phi(p, x, fz)
    # i: frozen at 0.3 (through the boundary), fluid at 0.5; the one at r_c and the one at 1.2 do not count
    assert phi[0] == pytest.approx(wc(0.3) ** 2 / (wc(0.3) ** 2 + wc(0.5) ** 2), rel=1e-14)
    assert phi[5] == 0.0


def _half_offset_interface(a=0.55, m=9):
    """Simple-cubic points at z = +-a/2, +-3a/2, ... (frozen below the plane
    z = 5, fluid above) with the probe particle on the plane between them at
    a lattice column: the configuration is mirror symmetric about the plane."""
    g = (np.arange(m) - m // 2) * a
    zs = (np.arange(m // 2) + 0.5) * a
    pts, fz = [], []
    for z in np.concatenate([-zs, zs]):
        for gx in g:
            for gy in g:
                pts.append([5.0 + gx, 5.0 + gy, 5.0 + z])
                fz.append(1 if z < 0 else 0)
    x = np.array([[5.0, 5.0, 5.0]] + pts)
    return x, np.array([0] + fz, np.uint8)


def test_phi_is_one_half_on_a_flat_interface(orc):
    """A fluid particle on the mirror plane of equal frozen and fluid
    half-lattices has phi = 1/2 exactly (the frozen and fluid sums are equal
    by symmetry); with the threshold phi_c = 0.5 it is not corrected."""
    x, fz = _half_offset_interface()
    phi = orc.phi(params(orc), x, fz)
    assert phi[0] == pytest.approx(0.5, abs=1e-14)
    # moving it 0.05 into the frozen side raises phi above 1/2, out of it lowers it
    for dz, sign in ((-0.05, 1.0), (0.05, -1.0)):
        y = x.copy()
        y[0, 2] += dz
        assert sign * (orc.phi(params(orc), y, fz)[0] - 0.5) > 0.01


# --------------------------------------------------------------------------
# Bin profiles
# --------------------------------------------------------------------------
def _sc_lattice(n_per_axis, box):
    a = box / n_per_axis
    g = (np.arange(n_per_axis) + 0.5) * a
    return np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_number_density_profile_of_a_lattice(orc, axis):
    """A 20^3 simple-cubic lattice in a 10^3 box (8000 particles, density 8):
    with 5 bins every bin holds 4 lattice planes of 400 points, so the bin
    density is 1600 / (10 * 10 * 2) = 8 exactly.  A bin index taken along
    another axis, a wrong bin volume or counting frozen particles breaks it;
    frozen particles added in bin 0 must not count."""
    x = _sc_lattice(20, L)
    extra = np.array([[0.2, 0.3, 0.4], [0.7, 0.1, 0.9]])  # frozen, in bin 0 along every axis
    xs = np.concatenate([x, extra])
    fz = np.concatenate([np.zeros(len(x), np.uint8), np.ones(2, np.uint8)])
    s = orc.System(params(orc, search=1), xs, np.zeros_like(xs), None, fz)
    np.testing.assert_allclose(s.profile(axis, 5, 0), 8.0, rtol=1e-14)
    # 8 bins of width 1.25: the planes at 0.25, 0.75 fall in bin 0, the one
    # exactly on the edge 1.25 opens bin 1 (1.25, 1.75, 2.25), and so on, so the
    # bins hold 2, 3, 2, 3, ... planes of 400 points
    planes = np.array([2, 3, 2, 3, 2, 3, 2, 3])
    np.testing.assert_allclose(s.profile(axis, 8, 0), planes * 400 / (L * L * L / 8), rtol=1e-14)


def test_velocity_and_temperature_profiles_of_a_prescribed_field(orc):
    """Velocities v = u(bin) + d_k on the 20^3 lattice, binned along y in 5
    bins: u(bin) = (0.1 b, -0.2, 0.05 b^2) and, inside each bin, deviations
    d_k = (+-0.3, +-0.3, +-0.3) with signs alternating so that they sum to
    zero per bin.  Then the bin means are u(bin) exactly and the peculiar
    temperature m |d|^2 / 3 = 0.09 m (m = 2 here).  Without the mean
    subtraction the kT profile would be m (0.09 + |u|^2 / 3) instead."""
    m = 2.0
    x = _sc_lattice(20, L)
    b = np.floor(x[:, 1] / L * 5).astype(int)
    u = np.stack([0.1 * b, np.full_like(b, -0.2, dtype=float), 0.05 * b**2], -1)
    # alternate the signs over the lattice columns: every y plane holds 200 of each
    sgn = np.where((np.floor(x[:, 0] / 0.5).astype(int) + np.floor(x[:, 2] / 0.5).astype(int)) % 2 == 0,
                   1.0, -1.0)
    d = 0.3 * np.stack([sgn, -sgn, sgn], -1)
    for q in range(5):
        assert abs(d[b == q].sum(axis=0)).max() < 1e-12
    v = u + d
    s = orc.System(params(orc, search=1, mass=m), x, v)
    ub = np.array([[0.1 * q, -0.2, 0.05 * q * q] for q in range(5)])
    for comp in range(3):
        np.testing.assert_allclose(s.profile(1, 5, 1 + comp), ub[:, comp], atol=1e-14)
    kt = s.profile(1, 5, 4)
    np.testing.assert_allclose(kt, m * 0.09, rtol=1e-12)
    no_sub = m * (0.09 + (ub**2).sum(-1) / 3.0)
    assert np.abs(kt - no_sub).max() > 0.005


def test_density_profile_of_the_many_body_density(orc):
    """Quantity 5 (mean many-body density per bin) on a simple-cubic lattice
    of spacing a = 0.55: every particle has rho = 6 w_rho(a) (only the six
    nearest neighbours are within r_d = 0.75; sqrt(2) a = 0.778 is not), so
    every bin holds 6 w_rho(0.55) = 6 * 15 / (2 pi 0.75^3) (1 - 0.55 / 0.75)^2."""
    a = 0.55
    n = 18
    box = n * a
    x = _sc_lattice(n, box)
    s = orc.System(orc.make_params(box=box, A=-40.0, B=25.0, gamma=4.5, rc=RC, rd=RD, search=1), x,
                   np.zeros_like(x))
    wr = 15.0 / (2.0 * np.pi * RD**3) * (1.0 - a / RD) ** 2
    np.testing.assert_allclose(s.profile(2, 3, 5), 6.0 * wr, rtol=1e-13)
