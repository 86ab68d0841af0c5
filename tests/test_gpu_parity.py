"""GPU parity of the HIP hot path against the FP64 oracle (needs an MI355X).

Bars (per the target of this path):
  * neighbour sets (r < r_c and r < r_d) bit-exact: count and set hash equal
  * FP64 form: per-particle forces within 1e-12 of the oracle, measured as
    max_i |F_i - F_i^oracle| / rms_k |F_k^oracle|; densities within 1e-12
    relative; positions and velocities within 1e-12 absolute after few steps
  * FP32-forces form: forces within 1e-5 by the same measure, densities within
    1e-5 relative
Every case prints its name first so that a failing run names it.
"""
import numpy as np
import pytest

import oracle
from paper_1903_10134_amd import workloads as W

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
FP32_TOL = 1e-5


@pytest.fixture(scope="module")
def mdpd():
    import torch
    assert torch.cuda.is_available()
    import paper_1903_10134_amd as m
    m.lib()
    return m


def say(*a):
    print("[case]", *a, flush=True)


def force_err(F, Fo):
    rms = np.sqrt(np.mean(np.sum(Fo * Fo, axis=1)))
    return float(np.abs(F - Fo).max() / rms) if F.size else 0.0


def rel_err(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)) if a.size else 0.0


def pdiff(x, xo, box):
    """Largest periodic (minimum-image) coordinate difference."""
    d = x - xo
    L = np.asarray(box, dtype=np.float64)
    d -= np.round(d / L) * L
    return float(np.abs(d).max()) if d.size else 0.0


def state_tols(precision, w, F_rms):
    """Position / velocity tolerances after one step implied by the force bar:
    a force error dF moves v by dt dF / m and x by dt^2 dF / (2 m)."""
    if precision == "fp64":
        return 1e-12, 1e-11
    dF = FP32_TOL * F_rms
    return 2.0 * (0.5 * w.dt ** 2 / w.mass * dF) + 1e-12, 2.0 * (w.dt / w.mass * dF) + 1e-11


def orc_params(w, search=0):
    return oracle.make_params(**w.param_kwargs(), search=search)


def dense_cluster(seed=4):
    """Background fluid plus 300 particles inside one cell: overflows the
    fixed-capacity neighbour list and exercises the direct-scan path.  Soft
    parameters and a short timestep keep the packed cell from exploding."""
    w = W.bulk(L=6.0, density=3.0, seed=seed, A=-4.0, B=2.0, gamma=0.45, dt=0.001)
    rng = np.random.default_rng(seed)
    extra = 2.0 + rng.random((300, 3)) * 0.9
    w.x = np.concatenate([w.x, extra])
    w.v = np.concatenate([w.v, rng.normal(size=(300, 3))])
    w.types = np.zeros(w.x.shape[0], np.int32)
    w.frozen = np.zeros(w.x.shape[0], np.uint8)
    w.name = "dense_cluster"
    return w


def mixed_types(seed=5):
    """Two types, a quarter of the particles frozen, walls off."""
    w = W.bulk(L=7.0, density=6.0, seed=seed)
    rng = np.random.default_rng(seed)
    w.types = (rng.random(w.n) < 0.3).astype(np.int32)
    w.frozen = (rng.random(w.n) < 0.25).astype(np.uint8)
    w.A = np.array([[-40.0, -30.0], [-30.0, -20.0]])
    w.B = np.array([[25.0, 22.0], [22.0, 28.0]])
    w.gamma = np.array([[4.5, 6.0], [6.0, 3.0]])
    w.g = (0.02, 0.0, -0.01)
    w.name = "mixed_types"
    return w


def small_cases():
    return {
        "bulk_L10_n6000": W.bulk(L=10.0, seed=0),
        "ragged_L7.3_n1000": W.bulk(L=7.3, n=1000, seed=1),
        "three_cells_L3.2": W.bulk(L=3.2, n=150, seed=2),
        "box_5x3.5x8.25": W.bulk(box=(5.0, 3.5, 8.25), n=900, seed=3),
        "two_cells_2x2.5x7": W.bulk(box=(2.0, 2.5, 7.0), n=210, seed=6),
        "slab_10x2x10": W.bulk(box=(10.0, 2.0, 10.0), n=1200, seed=7),
        "slab_8x8x2.5": W.bulk(box=(8.0, 8.0, 2.5), n=960, seed=8),
        "dense_cluster": dense_cluster(),
        "mixed_types": mixed_types(),
        # density 12: about 21 neighbours within r_d per particle, so most
        # FP32 near-r^2 rows run past their 16-entry head into the tail
        # area, and about 50 within r_c, so some rows overflow
        "dense_L6_rho12": W.bulk(L=6.0, density=12.0, seed=9),
    }


CASES = small_cases()


@pytest.mark.parametrize("name", list(CASES))
def test_neighbor_sets_bit_exact(mdpd, name):
    w = CASES[name]
    say("neighbor sets", name, w.n)
    s = mdpd.System(w)
    p = orc_params(w, search=0)
    for cut in (w.rc, w.rd, 0.5):
        c, h = s.neighbors(cut)
        co, ho = oracle.neighbors(p, w.x, cut)
        assert np.array_equal(c, co), (name, cut, int(np.sum(c != co)))
        assert np.array_equal(h, ho), (name, cut, int(np.sum(h != ho)))
    s.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("name", list(CASES))
def test_density_and_forces_step0_and_step1(mdpd, name, precision):
    w = CASES[name]
    say("step0/1", name, precision, w.n)
    prec = mdpd.FP64 if precision == "fp64" else mdpd.FP32_FORCES
    tol = FP64_TOL if precision == "fp64" else FP32_TOL
    s = mdpd.System(w, precision=prec)
    o = oracle.System(orc_params(w), w.x, w.v, w.types, w.frozen)
    F_rms = 0.0
    for step in (0, 1):
        if step:
            s.step(1)
            o.step(1)
        st = o.state()
        x, v, rho = s.state()
        F = s.forces()
        assert rel_err(rho, st["rho"]) < tol, (step, rel_err(rho, st["rho"]))
        assert force_err(F, st["F"]) < tol, (step, force_err(F, st["F"]))
        F_rms = max(F_rms, float(np.sqrt(np.mean(np.sum(st["F"] ** 2, axis=1)))))
        xtol, vtol = state_tols(precision, w, F_rms)
        assert pdiff(x, st["x"], w.box) < xtol, (step, pdiff(x, st["x"], w.box), xtol)
        assert np.abs(v - st["v"]).max() < vtol, (step, np.abs(v - st["v"]).max(), vtol)
    s.close()


@pytest.mark.parametrize("skin", [0.0, 0.1, 0.3, 0.6, 1.0])
def test_short_trajectory_fp64(mdpd, skin):
    """20 steps from the uniform-random start (hot: kT about 5), with list
    skins from none (a build every step) to one r_c (most skin rows then
    exceed their capacity and those particles take the direct cell scan):
    the pair sets are those of the oracle at every step, so the trajectory
    stays within rounding of it; every fourth step the sets at r_c and r_d
    are compared bit for bit."""
    w = CASES["bulk_L10_n6000"]
    say("trajectory 20 steps", w.name, "skin", skin)
    s = mdpd.System(w, skin=skin)
    o = oracle.System(orc_params(w), w.x, w.v)
    p = orc_params(w)
    for k in range(20):
        s.step(1)
        o.step(1)
        if k % 4 == 3:
            xo = o.state()["x"]
            for cut in (w.rc, w.rd):
                c, h = s.neighbors(cut)
                co, ho = oracle.neighbors(p, xo, cut)
                assert np.array_equal(c, co) and np.array_equal(h, ho), (k, cut)
    st = o.state()
    x, v, rho = s.state()
    assert pdiff(x, st["x"], w.box) < 1e-10
    assert np.abs(v - st["v"]).max() < 1e-9
    assert force_err(s.forces(), st["F"]) < 1e-9
    builds = s.list_builds()
    print(f"\nskin {skin}: {builds} list builds in 21 evaluations")
    if skin == 0.0:
        assert builds == 21
    if 0.3 <= skin <= 0.6:
        assert builds < 21
    s.close()


@pytest.mark.parametrize("name", ["bulk_L10_n6000", "mixed_types"])
def test_observables_match(mdpd, name):
    w = CASES[name]
    say("observables", name)
    s = mdpd.System(w)
    o = oracle.System(orc_params(w), w.x, w.v, w.types, w.frozen)
    for k in (0, 5):
        if k:
            s.step(k)
            o.step(k)
        a, b = s.observables(), o.observables()
        assert a["step"] == b["step"]
        for key in ("ke", "kT", "pressure", "epot", "mean_rho", "virial"):
            assert abs(a[key] - b[key]) <= 1e-11 * max(1.0, abs(b[key])), (key, a[key], b[key])
        for c, key in enumerate(("px", "py", "pz")):
            assert abs(a["momentum"][c] - b[key]) < 1e-9, key


def test_determinism_bitwise(mdpd):
    w = CASES["bulk_L10_n6000"]
    say("determinism", w.name)
    out = []
    for _ in range(2):
        s = mdpd.System(w, precision=mdpd.FP32_FORCES)
        s.step(10)
        x, v, rho = s.state()
        out.append((x, v, rho))
        s.close()
    for a, b in zip(*out):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("lanes", [1, 2, 8, 16])
def test_lane_splits_agree(mdpd, lanes):
    w = CASES["dense_cluster"]
    say("lanes", lanes)
    s = mdpd.System(w)
    for pss in range(3):
        s.set_lanes(pss, lanes)
    o = oracle.System(orc_params(w), w.x, w.v)
    s.step(2)
    o.step(2)
    st = o.state()
    assert force_err(s.forces(), st["F"]) < FP64_TOL
    c, h = s.neighbors(w.rc)
    co, ho = oracle.neighbors(orc_params(w), st["x"], w.rc)
    assert np.array_equal(c, co) and np.array_equal(h, ho)


@pytest.mark.parametrize("name", ["bulk_L10_n6000", "dense_cluster", "slab_10x2x10"])
def test_list_split_is_bitwise_neutral(mdpd, name):
    """Several wavefronts per cell of the list (pass 0 of set_lanes: the
    cell's particles dealt round robin) build the same rows, so the
    trajectory is bit for bit that of one wavefront per cell."""
    w = CASES[name]
    say("list split", name)
    ref = mdpd.System(w)
    ref.step(5)
    xr, vr, rr = ref.state()
    ref.close()
    for split in (2, 4, 8, 16):
        s = mdpd.System(w)
        s.set_lanes(0, split)
        s.step(5)
        x, v, rho = s.state()
        assert np.array_equal(x, xr) and np.array_equal(v, vr) and np.array_equal(rho, rr), split
        s.close()


def test_empty_and_single_particle(mdpd):
    say("empty / single")
    w = W.bulk(L=5.0, n=0)
    s = mdpd.System(w)
    s.step(3)
    o = s.observables()
    assert o["n"] == 0 and o["ke"] == 0.0
    s.close()
    w = W.bulk(L=5.0, n=1, seed=3)
    s = mdpd.System(w)
    s.step(3)
    x, v, _ = s.state()
    assert np.allclose(s.forces(), 0.0)
    assert np.allclose(v, w.v)
    s.close()


def test_invalid_inputs_are_rejected(mdpd):
    say("invalid inputs")
    w = W.bulk(L=5.0, n=50, seed=1)
    p = mdpd.make_params(**w.param_kwargs())
    bad = w.x.copy()
    bad[3, 1] = np.nan
    with pytest.raises(mdpd.MdpdError) as e:
        mdpd.mdpd_create(p, bad, w.v, w.types, w.frozen)
    assert e.value.status == -1
    bad = w.x.copy()
    bad[4, 0] = 2.5 * 5.0
    with pytest.raises(mdpd.MdpdError):
        mdpd.mdpd_create(p, bad, w.v, w.types, w.frozen)
    t = w.types.copy()
    t[0] = 3
    with pytest.raises(mdpd.MdpdError):
        mdpd.mdpd_create(p, w.x, w.v, t, w.frozen)
    small = mdpd.make_params(**{**w.param_kwargs(), "box": (1.99, 5.0, 5.0)})
    with pytest.raises(mdpd.MdpdError) as e:
        mdpd.mdpd_create(small, w.x * 0.39, w.v, w.types, w.frozen)
    assert e.value.status == -1
    p2 = mdpd.make_params(**{**w.param_kwargs(), "rd": 1.5})
    with pytest.raises(mdpd.MdpdError):
        mdpd.mdpd_create(p2, w.x, w.v, w.types, w.frozen)
    p3 = mdpd.make_params(**{**w.param_kwargs(), "wall_model": 1, "phi_c": -0.1})
    with pytest.raises(mdpd.MdpdError) as e:
        mdpd.mdpd_create(p3, w.x, w.v, w.types, w.frozen)
    assert e.value.status == -1


def test_nonfinite_state_is_reported(mdpd):
    """A non-finite half-step velocity planted in a checkpoint (the layout of
    mdpd_save_checkpoint: header and parameters, then 256-byte aligned fields
    x, v, F, predicted x, predicted half-step v, ...) makes the next
    mdpd_step return MDPD_E_NONFINITE; a velocity so large that the first
    predicted move leaves the box makes mdpd_create return it."""
    import ctypes
    w = W.bulk(L=5.0, n=600, seed=8)
    say("non-finite state")
    s = mdpd.System(w)
    s.step(2)
    buf = s.save_checkpoint()
    al = lambda b: (b + 255) // 256 * 256  # noqa: E731
    head = al(64 + ctypes.sizeof(mdpd.Params))
    off = head + 4 * al(24 * w.n)
    bad = buf.copy()
    bad[off:off + 8] = np.frombuffer(np.array([np.nan]).tobytes(), np.uint8)
    s.load_checkpoint(bad)
    with pytest.raises(mdpd.MdpdError) as e:
        s.step(1)
    assert e.value.status == -4
    s.load_checkpoint(buf)  # the good state steps on
    s.step(1)
    s.close()
    v = w.v.copy()
    v[7] = (1e200, 0.0, 0.0)
    p = mdpd.make_params(**w.param_kwargs())
    with pytest.raises(mdpd.MdpdError) as e:
        mdpd.mdpd_create(p, w.x, v, w.types, w.frozen)
    assert e.value.status == -4


def test_device_inputs_equal_host_inputs(mdpd):
    import torch
    w = CASES["ragged_L7.3_n1000"]
    say("device inputs")
    a = mdpd.System(w)
    b = mdpd.System(w, device_inputs=True, stream=torch.cuda.current_stream())
    a.step(3)
    b.step(3)
    for u, v in zip(a.state(), b.state()):
        assert np.array_equal(u, v)


# ---------------------------------------------------------------------------
# Full size: 1,053,696 particles (56^3 cells at number density 6), the launch
# configuration the benchmark times.
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def full():
    w = W.bulk(L=56.0, seed=0)
    o = oracle.System(orc_params(w, search=1), w.x, w.v)
    st0 = o.state()
    o.step(1)
    st1 = o.state()
    return w, st0, st1


def test_full_size_neighbor_sets(mdpd, full):
    w, st0, _ = full
    say("full size neighbor sets", w.n)
    s = mdpd.System(w, precision=mdpd.FP32_FORCES)
    p = orc_params(w, search=1)
    for cut in (w.rc, w.rd):
        c, h = s.neighbors(cut)
        co, ho = oracle.neighbors(p, w.x, cut)
        assert np.array_equal(c, co) and np.array_equal(h, ho), cut


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_full_size_forces(mdpd, full, precision):
    w, st0, st1 = full
    say("full size forces", precision, w.n)
    prec = mdpd.FP64 if precision == "fp64" else mdpd.FP32_FORCES
    tol = FP64_TOL if precision == "fp64" else FP32_TOL
    s = mdpd.System(w, precision=prec)
    assert force_err(s.forces(), st0["F"]) < tol
    s.step(1)
    x, v, rho = s.state()
    assert force_err(s.forces(), st1["F"]) < tol
    assert rel_err(rho, st1["rho"]) < tol
    F_rms = float(np.sqrt(np.mean(np.sum(st0["F"] ** 2, axis=1))))
    xtol, vtol = state_tols(precision, w, F_rms)
    assert pdiff(x, st1["x"], w.box) < xtol
    assert np.abs(v - st1["v"]).max() < 2 * vtol


# ---------------------------------------------------------------------------
# Wall treatment (boundary volume fraction + predictor-corrector) and profiles
# ---------------------------------------------------------------------------
def small_channel(seed=7):
    """Channel of the Poiseuille set-up at a size the oracle steps quickly."""
    return W.channel(Lx=8.0, Ly=6.0, Lz=8.0, wall=2.0, seed=seed, gx=0.05)


@pytest.mark.parametrize("skin", [0.0, 0.3])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_wall_corrector_parity(mdpd, precision, skin):
    w = small_channel()
    say("walls", precision, w.n, "skin", skin)
    prec = mdpd.FP64 if precision == "fp64" else mdpd.FP32_FORCES
    s = mdpd.System(w, precision=prec, skin=skin)
    o = oracle.System(orc_params(w), w.x, w.v, w.types, w.frozen)
    total = 0
    for k in range(12):
        s.step(1)
        o.step(1)
        a, b = s.observables(), o.observables()
        assert a["ncorr_last"] == b["ncorr_last"], (k, a["ncorr_last"], b["ncorr_last"])
        total += b["ncorr_last"]
    st = o.state()
    x, v, rho = s.state()
    F_rms = float(np.sqrt(np.mean(np.sum(st["F"] ** 2, axis=1))))
    if precision == "fp64":
        assert pdiff(x, st["x"], w.box) < 1e-10
        assert force_err(s.forces(), st["F"]) < 1e-10
    else:
        assert pdiff(x, st["x"], w.box) < 1e-4
        assert force_err(s.forces(), st["F"]) < 1e-3
    assert a["ncorr_total"] == b["ncorr_total"] == total
    assert total > 0, "the case should exercise the corrector"


@pytest.mark.parametrize("eta", [1.0, 0.4])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_dissipation_control_parity(mdpd, precision, eta):
    """Control of the effective fluid-solid dissipation (diss_ctrl = eta,
    diss_rho = 6) on the walled channel: forces at creation, then equal
    corrector counts at every step and the state after 12 steps, against the
    oracle.  The control must change the near-wall forces (not a no-op)."""
    w = small_channel(seed=11)
    w.diss_ctrl, w.diss_rho = eta, 6.0
    say("dissipation control", precision, eta, w.n)
    prec = mdpd.FP64 if precision == "fp64" else mdpd.FP32_FORCES
    s = mdpd.System(w, precision=prec)
    o = oracle.System(orc_params(w), w.x, w.v, w.types, w.frozen)
    F0 = o.state()["F"]
    tol0 = 1e-12 if precision == "fp64" else 2e-5
    assert force_err(s.forces(), F0) < tol0
    w_off = small_channel(seed=11)
    o_off = oracle.System(orc_params(w_off), w_off.x, w_off.v, w_off.types, w_off.frozen)
    assert force_err(o_off.state()["F"], F0) > 1e-3, "the control should change the near-wall forces"
    total = 0
    for k in range(12):
        s.step(1)
        o.step(1)
        a, b = s.observables(), o.observables()
        assert a["ncorr_last"] == b["ncorr_last"], (k, a["ncorr_last"], b["ncorr_last"])
        total += b["ncorr_last"]
    st = o.state()
    x, v, rho = s.state()
    if precision == "fp64":
        assert pdiff(x, st["x"], w.box) < 1e-10
        assert force_err(s.forces(), st["F"]) < 1e-10
    else:
        assert pdiff(x, st["x"], w.box) < 1e-4
        assert force_err(s.forces(), st["F"]) < 1e-3
    assert total > 0, "the case should exercise the corrector"


def test_profiles_match_oracle(mdpd):
    w = small_channel(seed=8)
    say("profiles")
    s = mdpd.System(w)
    o = oracle.System(orc_params(w), w.x, w.v, w.types, w.frozen)
    s.step(5)
    o.step(5)
    for axis in (0, 1):
        for q in range(6):
            pa, pb = s.profile(axis, 8, q), o.profile(axis, 8, q)
            assert np.allclose(pa, pb, rtol=1e-9, atol=1e-10), (axis, q, pa, pb)


@pytest.mark.parametrize("case,prec,skin", [("bulk_L10_n6000", "fp32", 0.0), ("dense_cluster", "fp64", 0.0),
                                            ("small_channel", "fp64", 0.0), ("small_channel", "fp32", 0.0),
                                            ("slip_channel", "fp32", 0.0), ("bulk_L10_n6000", "fp32", 0.3),
                                            ("small_channel", "fp64", 0.3)])
def test_checkpoint_resume_bitwise(mdpd, case, prec, skin):
    """A checkpoint loaded into a fresh system continues bit for bit: state,
    forces, observables and neighbour sets after more steps."""
    if case == "slip_channel":
        w = small_channel(seed=9)
        w.wall_slip = 0.75
    else:
        w = small_channel() if case == "small_channel" else CASES[case]
    p = mdpd.FP32_FORCES if prec == "fp32" else mdpd.FP64
    say("checkpoint", case, prec, "skin", skin)
    a = mdpd.System(w, precision=p, skin=skin)
    a.step(7)
    buf = a.save_checkpoint()
    obs0 = a.observables()
    a.step(9)
    b = mdpd.System(w, precision=p, skin=skin)  # same parameters, fresh state at step 0
    b.load_checkpoint(buf)
    assert b.observables() == obs0
    b.step(9)
    for u, v in zip(a.state(), b.state()):
        assert np.array_equal(u, v)
    assert np.array_equal(a.forces(), b.forces())
    assert a.observables() == b.observables()
    for cut in (w.rd, w.rc):
        ca, ha = a.neighbors(cut)
        cb, hb = b.neighbors(cut)
        assert np.array_equal(ca, cb) and np.array_equal(ha, hb)
    a.close()
    b.close()


def test_checkpoint_rejects_other_systems(mdpd):
    w = CASES["bulk_L10_n6000"]
    a = mdpd.System(w)
    buf = a.save_checkpoint()
    c = mdpd.System(w, precision=mdpd.FP32_FORCES)  # other parameters
    with pytest.raises(mdpd.MdpdError):
        c.load_checkpoint(buf)
    with pytest.raises(mdpd.MdpdError):
        a.load_checkpoint(buf[:100])
    bad = buf.copy()
    bad[0] ^= 1
    with pytest.raises(mdpd.MdpdError):
        a.load_checkpoint(bad)
    a.load_checkpoint(buf)  # the original still loads
    a.close()
    c.close()


def test_observables_deterministic_with_list_overflow(mdpd):
    """dense_cluster overflows the neighbour-list rows; the energy and virial
    shares of those particles are reduced in a fixed order."""
    w = CASES["dense_cluster"]
    outs = []
    for _ in range(2):
        s = mdpd.System(w, precision=mdpd.FP32_FORCES)
        s.step(3)
        outs.append(s.observables())
        s.close()
    assert outs[0] == outs[1]
