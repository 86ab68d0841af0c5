"""Pins of the oracle's forward-mode derivative (orc_tangent).

The derivative of the loss of a trajectory along a direction in the inputs
(initial positions and velocities, the pair tables A, B, gamma) is checked
against central finite differences of plain oracle runs (orc_step and
orc_observables, which share no derivative code), and against exact
invariances: a uniform translation changes nothing, a uniform velocity boost
shifts the mean velocity by itself, and pairwise antisymmetric forces keep
the mean fluid velocity independent of the force parameters.  CPU only.
"""
import numpy as np
import pytest

from paper_1903_10134_amd import workloads as W

RHO, PRES, VX = (1.0, 0.0, 0.0), (0.0, 1.0, 0.0), (0.0, 0.0, 1.0)


def _case(kind):
    w = W.bulk(L=6.0, density=6.0, seed=3)
    kw = w.param_kwargs()
    kw.pop("precision", None)
    types = np.zeros(w.x.shape[0], np.int32)
    frozen = np.zeros(w.x.shape[0], np.uint8)
    rng = np.random.default_rng(11)
    if kind == "two_types":
        types = rng.integers(0, 2, w.x.shape[0]).astype(np.int32)
        kw["A"] = np.array([[-40.0, -30.0], [-30.0, -35.0]])
        kw["B"] = np.array([[25.0, 24.0], [24.0, 26.0]])
        kw["gamma"] = np.array([[4.5, 4.0], [4.0, 5.0]])
    elif kind == "frozen":
        frozen = (rng.random(w.x.shape[0]) < 0.15).astype(np.uint8)
    elif kind == "walls":
        # a small driven channel with the bounce-back corrector: its events
        # are held fixed, so central differences with small steps see the
        # same events as the tangent
        w = W.channel(Lx=6.0, Ly=4.0, Lz=6.0, wall=1.5, seed=3, gx=0.05)
        kw = w.param_kwargs()
        types, frozen = w.types, w.frozen
    elif kind == "walls_dc":
        # the same channel with the fluid-solid dissipation control (its
        # factor s_i depends on the positions and has a tangent of its own)
        w = W.channel(Lx=6.0, Ly=4.0, Lz=6.0, wall=1.5, seed=3, gx=0.05)
        w.diss_ctrl, w.diss_rho = 0.8, 6.0
        kw = w.param_kwargs()
        types, frozen = w.types, w.frozen
    return w, kw, types, frozen


def _fd(orc, kw, x, v, types, frozen, nsteps, wts, avg, h, shift):
    def f(e):
        kw2, x0, v0 = shift(dict(kw), x.copy(), v.copy(), e)
        return orc.loss(orc.make_params(**kw2), x0, v0, types, frozen, nsteps, wts, avg)
    return (f(h) - f(-h)) / (2.0 * h)


def _close(dL, fd, rel, floor):
    return abs(dL - fd) <= rel * abs(fd) + floor


@pytest.mark.parametrize("kind", ["one_type", "two_types", "frozen", "walls", "walls_dc"])
@pytest.mark.parametrize("nsteps,avg", [(0, False), (4, False), (4, True)])
def test_tangent_matches_finite_differences(orc, kind, nsteps, avg):
    w, kw, types, frozen = _case(kind)
    p = orc.make_params(**kw)
    n = w.x.shape[0]
    T = np.atleast_2d(kw["A"]).shape[0]
    rng = np.random.default_rng(nsteps + 7 * avg)
    dx = rng.standard_normal((n, 3))
    dv = rng.standard_normal((n, 3))
    # a symmetric direction in the tables: all entries of the (0, T-1) pair
    E = np.zeros((T, T))
    E[0, T - 1] = E[T - 1, 0] = 1.0

    def table(name):
        return lambda k, x, v, e: ({**k, name: np.atleast_2d(k[name]) + e * E}, x, v)

    dirs = {
        "A": (dict(dA=E.ravel()), table("A"), 1e-6),
        "B": (dict(dB=E.ravel()), table("B"), 1e-6),
        "gamma": (dict(dgamma=E.ravel()), table("gamma"), 1e-6),
        "x0": (dict(dx0=dx), lambda k, x, v, e: (k, x + e * dx, v), 1e-7),
        "v0": (dict(dv0=dv), lambda k, x, v, e: (k, x, v + e * dv), 1e-6),
    }
    for wts in (RHO, PRES) + ((VX,) if kind == "walls_dc" else ()):
        for name, (kwargs, shift, h) in dirs.items():
            L, dL = orc.tangent(p, w.x, w.v, types, frozen, nsteps, wts, avg, **kwargs)
            fd = _fd(orc, kw, w.x, w.v, types, frozen, nsteps, wts, avg, h, shift)
            scale = 1.0 if wts is RHO else 100.0
            assert _close(dL, fd, 2e-6, 1e-7 * scale), (wts, name, dL, fd)


def test_tangent_loss_value_is_the_forward_loss(orc):
    w, kw, types, frozen = _case("frozen")
    p = orc.make_params(**kw)
    for nsteps, avg in ((0, False), (3, False), (3, True)):
        for wts in (RHO, PRES, VX, (0.3, -0.01, 2.0)):
            L, _ = orc.tangent(p, w.x, w.v, types, frozen, nsteps, wts, avg)
            assert L == pytest.approx(orc.loss(p, w.x, w.v, types, frozen, nsteps, wts, avg), rel=1e-13,
                                      abs=1e-13)


def test_uniform_translation_changes_nothing(orc):
    w, kw, types, frozen = _case("frozen")
    p = orc.make_params(**kw)
    d = np.tile([0.3, -1.1, 0.7], (w.x.shape[0], 1))
    for wts in (RHO, PRES, VX):
        _, dL = orc.tangent(p, w.x, w.v, types, frozen, 4, wts, False, dx0=d)
        assert abs(dL) < 1e-9


def test_galilean_boost_and_momentum(orc):
    w, kw, types, frozen = _case("two_types")
    p = orc.make_params(**kw)
    n = w.x.shape[0]
    boost = np.tile([1.0, 0.0, 0.0], (n, 1))
    _, d_vx = orc.tangent(p, w.x, w.v, types, frozen, 4, VX, False, dv0=boost)
    _, d_rho = orc.tangent(p, w.x, w.v, types, frozen, 4, RHO, False, dv0=boost)
    assert d_vx == pytest.approx(1.0, abs=1e-12)
    assert abs(d_rho) < 1e-10
    T = 2
    for name in ("dA", "dB", "dgamma"):
        _, d = orc.tangent(p, w.x, w.v, types, frozen, 4, VX, True, **{name: np.ones(T * T)})
        assert abs(d) < 1e-12


def test_tangent_with_wall_events(orc):
    """The walled case has corrector events within the differentiated steps,
    its loss value is the forward loss, and reflecting walls (wall_slip > 0,
    whose normal would need a derivative) are refused."""
    w, kw, types, frozen = _case("walls")
    p = orc.make_params(**kw)
    s = orc.System(p, w.x, w.v, types, frozen)
    s.step(4)
    assert s.observables()["ncorr_total"] > 0
    L, _ = orc.tangent(p, w.x, w.v, types, frozen, 4, RHO, False)
    assert L == pytest.approx(orc.loss(p, w.x, w.v, types, frozen, 4, RHO, False), rel=1e-13, abs=1e-13)
    q = orc.make_params(**{**kw, "wall_slip": 0.5})
    with pytest.raises(ValueError):
        orc.tangent(q, w.x, w.v, types, frozen, 2, RHO)
