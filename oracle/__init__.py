"""FP64 CPU oracle of the many-body DPD timestep (test infrastructure only).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark use
this package.  It wraps ``mdpd_oracle.c`` (plain C, FP64, O(N^2) brute-force
neighbour search plus an equivalent naive linked-cell search) through ctypes.
It shares no code with the GPU library and never imports it.

Every function cites the passage of the paper it follows in the C source; the
pins that tie it to something other than itself live in
``tests/test_oracle_pins.py``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mdpd_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
MAXT = 8


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP contraction off, OpenMP over particles)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
             "-fPIC", "-shared", "-D_GNU_SOURCE", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class Params(ctypes.Structure):
    _fields_ = [
        ("L", ctypes.c_double * 3),
        ("rc", ctypes.c_double), ("rd", ctypes.c_double), ("kT", ctypes.c_double),
        ("dt", ctypes.c_double), ("mass", ctypes.c_double),
        ("g", ctypes.c_double * 3),
        ("phi_c", ctypes.c_double),
        ("wall_slip", ctypes.c_double),
        ("A", ctypes.c_double * (MAXT * MAXT)),
        ("B", ctypes.c_double * (MAXT * MAXT)),
        ("gamma", ctypes.c_double * (MAXT * MAXT)),
        ("seed", ctypes.c_uint32),
        ("ntypes", ctypes.c_int32),
        ("wall_model", ctypes.c_int32),
        ("search", ctypes.c_int32),
        ("diss_ctrl", ctypes.c_double),
        ("diss_rho", ctypes.c_double),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        P = ctypes.POINTER
        d, u8, i32, i64, u64 = (ctypes.c_double, ctypes.c_uint8, ctypes.c_int32,
                                ctypes.c_int64, ctypes.c_uint64)
        L.orc_threefry2x32_20.argtypes = [P(ctypes.c_uint32), P(ctypes.c_uint32), P(ctypes.c_uint32)]
        L.orc_theta.argtypes = [ctypes.c_uint32] * 4
        L.orc_theta.restype = d
        L.orc_theta_many.argtypes = [ctypes.c_uint32, ctypes.c_uint32, i64, P(ctypes.c_uint32),
                                     P(ctypes.c_uint32), P(d)]
        L.orc_mix64.argtypes = [u64]
        L.orc_mix64.restype = u64
        L.orc_wrap.argtypes = [d, d]
        L.orc_wrap.restype = d
        L.orc_w_rho.argtypes = [d, d]
        L.orc_w_rho.restype = d
        L.orc_neighbors.argtypes = [P(Params), i64, P(d), d, P(i64), P(u64)]
        L.orc_density.argtypes = [P(Params), i64, P(d), P(d)]
        L.orc_phi.argtypes = [P(Params), i64, P(d), P(u8), P(d)]
        L.orc_diss_scale.argtypes = [P(Params), i64, P(d), P(u8), P(d)]
        L.orc_forces.argtypes = [P(Params), i64, P(d), P(d), P(i32), P(u8), P(d), ctypes.c_uint32,
                                 P(d), P(d), P(d)]
        L.orc_create.argtypes = [P(Params), i64, P(d), P(d), P(i32), P(u8)]
        L.orc_create.restype = ctypes.c_void_p
        L.orc_step.argtypes = [ctypes.c_void_p, i64]
        L.orc_get.argtypes = [ctypes.c_void_p, P(d), P(d), P(d), P(d), P(d)]
        L.orc_observables.argtypes = [ctypes.c_void_p, P(d)]
        L.orc_profile.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, P(d)]
        L.orc_destroy.argtypes = [ctypes.c_void_p]
        L.orc_num_threads.argtypes = []
        L.orc_num_threads.restype = ctypes.c_int
        L.orc_set_num_threads.argtypes = [ctypes.c_int]
        L.orc_set_num_threads.restype = None
        L.orc_current_step.argtypes = [ctypes.c_void_p]
        L.orc_current_step.restype = ctypes.c_uint32
        L.orc_tangent.argtypes = [P(Params), i64, P(d), P(d), P(i32), P(u8), P(d), P(d), P(d), P(d), P(d),
                                  i64, P(d), ctypes.c_int, P(d)]
        L.orc_tangent.restype = ctypes.c_int
        L.orc_stress.argtypes = [ctypes.c_void_p, P(d)]
        _lib = L
    return _lib


def _ptr(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def make_params(box, A, B, gamma, rc=1.0, rd=0.75, kT=1.0, dt=0.01, mass=1.0, g=(0.0, 0.0, 0.0),
                seed=0, wall_model=0, phi_c=0.5, search=0, wall_slip=0.0, diss_ctrl=0.0,
                diss_rho=0.0) -> Params:
    """Build the oracle's parameter block.  A, B, gamma: scalars or T x T.
    diss_ctrl, diss_rho: the dissipation control (eta, rho_f) of reading R6."""
    A = np.atleast_2d(np.asarray(A, dtype=np.float64))
    B = np.atleast_2d(np.asarray(B, dtype=np.float64))
    G = np.atleast_2d(np.asarray(gamma, dtype=np.float64))
    T = A.shape[0]
    if B.shape != (T, T) or G.shape != (T, T) or A.shape != (T, T) or not 1 <= T <= MAXT:
        raise ValueError("A, B, gamma must be T x T with 1 <= T <= 8")
    p = Params()
    p.L[:] = [float(b) for b in (box if np.ndim(box) else (box, box, box))]
    p.rc, p.rd, p.kT, p.dt, p.mass = rc, rd, kT, dt, mass
    p.g[:] = [float(v) for v in g]
    p.phi_c = phi_c
    p.wall_slip = float(wall_slip)
    p.diss_ctrl = float(diss_ctrl)
    p.diss_rho = float(diss_rho)
    for name, M in (("A", A), ("B", B), ("gamma", G)):
        arr = getattr(p, name)
        for a in range(T):
            for b in range(T):
                arr[a * T + b] = M[a, b]
    p.seed = int(seed) & 0xFFFFFFFF
    p.ntypes = T
    p.wall_model = int(wall_model)
    p.search = int(search)
    return p


def num_threads() -> int:
    """Threads the oracle's OpenMP loops use."""
    return int(lib().orc_num_threads())


def set_num_threads(n: int) -> None:
    """Set the threads of the oracle's OpenMP loops (for timing on one core)."""
    lib().orc_set_num_threads(int(n))


def threefry2x32_20(ctr, key):
    c = (ctypes.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (ctypes.c_uint32 * 2)()
    lib().orc_threefry2x32_20(c, k, o)
    return int(o[0]), int(o[1])


def theta(seed, step, i, j) -> float:
    return float(lib().orc_theta(seed & 0xFFFFFFFF, step & 0xFFFFFFFF, i, j))


def theta_many(seed, step, i, j):
    i = np.ascontiguousarray(np.asarray(i, dtype=np.uint32))
    j = np.ascontiguousarray(np.asarray(j, dtype=np.uint32))
    out = np.zeros(i.shape[0])
    lib().orc_theta_many(seed & 0xFFFFFFFF, step & 0xFFFFFFFF, i.shape[0], _ptr(i, ctypes.c_uint32),
                         _ptr(j, ctypes.c_uint32), _ptr(out, ctypes.c_double))
    return out


def mix64(z: int) -> int:
    return int(lib().orc_mix64(int(z) & 0xFFFFFFFFFFFFFFFF))


def w_rho(r: float, rd: float) -> float:
    return float(lib().orc_w_rho(r, rd))


def wrap(x: float, L: float) -> float:
    return float(lib().orc_wrap(x, L))


def _c3(x):
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(-1, 3))


def neighbors(p: Params, x, cutoff):
    x = _c3(x)
    n = x.shape[0]
    cnt = np.zeros(n, dtype=np.int64)
    h = np.zeros(n, dtype=np.uint64)
    lib().orc_neighbors(ctypes.byref(p), n, _ptr(x, ctypes.c_double), float(cutoff),
                        _ptr(cnt, ctypes.c_int64), _ptr(h, ctypes.c_uint64))
    return cnt, h


def density(p: Params, x):
    x = _c3(x)
    rho = np.zeros(x.shape[0])
    lib().orc_density(ctypes.byref(p), x.shape[0], _ptr(x, ctypes.c_double), _ptr(rho, ctypes.c_double))
    return rho


def phi(p: Params, x, frozen):
    x = _c3(x)
    fz = np.ascontiguousarray(np.asarray(frozen, dtype=np.uint8))
    out = np.zeros(x.shape[0])
    lib().orc_phi(ctypes.byref(p), x.shape[0], _ptr(x, ctypes.c_double), _ptr(fz, ctypes.c_uint8),
                  _ptr(out, ctypes.c_double))
    return out


def diss_scale(p: Params, x, frozen):
    """Dissipation-control factors s_i of the fluid-solid pairs (reading R6)."""
    x = _c3(x)
    fz = np.ascontiguousarray(np.asarray(frozen, dtype=np.uint8))
    out = np.zeros(x.shape[0])
    lib().orc_diss_scale(ctypes.byref(p), x.shape[0], _ptr(x, ctypes.c_double), _ptr(fz, ctypes.c_uint8),
                         _ptr(out, ctypes.c_double))
    return out


def forces(p: Params, x, vh, types, frozen, rho, step):
    """Pair + body forces on fluid particles; returns (F, virial, epair)."""
    x = _c3(x)
    vh = _c3(vh)
    n = x.shape[0]
    t = np.ascontiguousarray(np.asarray(types, dtype=np.int32))
    fz = np.ascontiguousarray(np.asarray(frozen, dtype=np.uint8))
    rho = np.ascontiguousarray(np.asarray(rho, dtype=np.float64))
    F = np.zeros((n, 3))
    vir = ctypes.c_double()
    ep = ctypes.c_double()
    lib().orc_forces(ctypes.byref(p), n, _ptr(x, ctypes.c_double), _ptr(vh, ctypes.c_double),
                     _ptr(t, ctypes.c_int32), _ptr(fz, ctypes.c_uint8), _ptr(rho, ctypes.c_double),
                     int(step) & 0xFFFFFFFF, _ptr(F, ctypes.c_double), ctypes.byref(vir), ctypes.byref(ep))
    return F, vir.value, ep.value


OBS_NAMES = ("step", "ke", "kT", "pressure", "px", "py", "pz", "epot", "mean_rho",
             "ncorr_last", "ncorr_total", "virial")


class System:
    """An oracle system advanced with velocity-Verlet in the order of Alg. 1."""

    def __init__(self, p: Params, x, v, types=None, frozen=None):
        x = _c3(x)
        v = _c3(v)
        n = x.shape[0]
        t = np.zeros(n, np.int32) if types is None else np.asarray(types, np.int32)
        fz = np.zeros(n, np.uint8) if frozen is None else np.asarray(frozen, np.uint8)
        t = np.ascontiguousarray(t)
        fz = np.ascontiguousarray(fz)
        self.n = n
        self.p = p
        self._h = lib().orc_create(ctypes.byref(p), n, _ptr(x, ctypes.c_double),
                                   _ptr(v, ctypes.c_double), _ptr(t, ctypes.c_int32),
                                   _ptr(fz, ctypes.c_uint8))

    def step(self, nsteps: int = 1):
        lib().orc_step(self._h, int(nsteps))

    @property
    def current_step(self) -> int:
        return int(lib().orc_current_step(self._h))

    def state(self):
        n = self.n
        x, v, F, vh = (np.zeros((n, 3)) for _ in range(4))
        rho = np.zeros(n)
        d = ctypes.c_double
        lib().orc_get(self._h, _ptr(x, d), _ptr(v, d), _ptr(F, d), _ptr(rho, d), _ptr(vh, d))
        return {"x": x, "v": v, "F": F, "rho": rho, "vh": vh}

    def observables(self) -> dict:
        out = np.zeros(12)
        lib().orc_observables(self._h, _ptr(out, ctypes.c_double))
        return dict(zip(OBS_NAMES, out.tolist()))

    def stress(self):
        """Pressure tensor (xx, yy, zz, xy, xz, yz), brute-force pair sum."""
        out = np.zeros(6)
        lib().orc_stress(self._h, _ptr(out, ctypes.c_double))
        return out

    def profile(self, axis: int, nbins: int, quantity: int):
        out = np.zeros(nbins)
        lib().orc_profile(self._h, axis, nbins, quantity, _ptr(out, ctypes.c_double))
        return out

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_destroy(h)
            self._h = None


def _opt(a, shape):
    if a is None:
        return None
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(shape))


def tangent(p: Params, x0, v0, types, frozen, nsteps, w, avg=False, dx0=None, dv0=None, dA=None, dB=None,
            dgamma=None):
    """Loss L and its derivative dL along the direction (dx0, dv0, dA, dB,
    dgamma) by forward-mode differentiation of the trajectory (with walls:
    bounce-back only, the corrector's decisions held fixed).
    L = w0 mean_fluid(rho) + w1 P + w2 mean_fluid(v_x) of the final state,
    or its mean over steps 1..nsteps when avg."""
    x0 = _c3(x0)
    v0 = _c3(v0)
    n = x0.shape[0]
    T = p.ntypes
    t = np.ascontiguousarray(np.asarray(types, np.int32))
    fz = np.ascontiguousarray(np.asarray(frozen, np.uint8))
    d = ctypes.c_double
    arrs = [_opt(dx0, (n, 3)), _opt(dv0, (n, 3))] + [_opt(q, (T * T,)) for q in (dA, dB, dgamma)]
    ptrs = [None if a is None else _ptr(a, d) for a in arrs]
    wv = np.ascontiguousarray(np.asarray(w, dtype=np.float64))
    out = np.zeros(2)
    rc = lib().orc_tangent(ctypes.byref(p), n, _ptr(x0, d), _ptr(v0, d), _ptr(t, ctypes.c_int32),
                           _ptr(fz, ctypes.c_uint8), *ptrs, int(nsteps), _ptr(wv, d), 1 if avg else 0,
                           _ptr(out, d))
    if rc != 0:
        raise ValueError("orc_tangent: needs bounce-back walls or none, no dissipation control, and "
                         "nsteps >= 1 with avg")
    return float(out[0]), float(out[1])


def loss(p: Params, x0, v0, types, frozen, nsteps, w, avg=False):
    """The same loss from plain orc_step runs and orc_observables (no
    derivative code involved): the finite-difference reference."""
    s = System(p, x0, v0, types, frozen)

    def one():
        o = s.observables()
        st = s.state()
        fl = np.asarray(frozen, bool) == 0
        nf = max(int(fl.sum()), 1)
        return w[0] * o["mean_rho"] + w[1] * o["pressure"] + w[2] * st["v"][fl, 0].sum() / nf

    if not avg:
        s.step(nsteps)
        return one()
    acc = 0.0
    for _ in range(nsteps):
        s.step(1)
        acc += one()
    return acc / nsteps
